"""Parity at the clustered workload's and the serving workload's full sizes.

Clustered (Algorithm 4; clustering-based protocol, steps 5 and 8): 10M x 96
int8 points in 16,384 Zipf-sized clusters plus a 100,000-point stash, 32
queries per launch, 64 clusters per query, N = 8192, L = 3, on a context
created as the benchmark creates it.  Checked:
  * phase 1 (centre distances) and phase 2 (the per-query chunk lists) decrypt
    to the true squared distance at every slot of every output row, for all
    32 queries; the selected clusters are the 64 closest in the clear;
  * sampled phase-1 and phase-2 rows against the oracle on uniform residue
    inputs (server shares in full, ciphertext coefficients at sampled
    positions): a chunk shared by several queries, a stash chunk, the last
    (padding) chunk, and the shortest and longest per-query lists.

Serving (continuous batching over three resident databases: 100K x 128
uint8, 1M x 96 int8 and the clustered index): a short Poisson trace; every
request's outputs equal the same request served alone, and decrypt to the
true distances at every slot of every row.
"""
import numpy as np
import pytest

import oracle
import synthdata

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

U = 64


def _i64(x):
    if x.dtype == torch.uint32:
        return x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return x.view(torch.int64)


def _digit_ctx(nat, stage, w):
    params = nat.sanns_params_derive(w.N, w.L, w.t_bits)
    params.flags |= nat.SANNS_FLAG_DIGIT_DB
    return stage.Context(params=params)


def _encrypt(stage, ctx, queries, seed, dev):
    Qn, d = queries.shape
    sk = torch.as_tensor(synthdata.gen_secret(ctx.N, seed)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, ctx.N, Qn * d, seed + 1)
    e = synthdata.gen_cbd_error(ctx.N, Qn * d, seed + 1)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    torch.cuda.synchronize()
    return sk, ct


def _closed_form(stage, ctx, sk, out, share, qrows, chunks, slot_map, pts, dev, batch=48):
    """client + server = ||q - p||^2 at every real slot of every row (exact
    int32 sums on the device) and ||q||^2 at padding slots (a zero point).
    qrows: [M][d] the query of each row; chunks: [M] its chunk.  Returns the
    number of real slots checked."""
    M, N, t = out.shape[0], ctx.N, ctx.t
    qn2 = (qrows.astype(np.int64) ** 2).sum(axis=1) % t
    client = stage.decrypt_shares(ctx, sk, out.contiguous(),
                                  torch.as_tensor(qn2.astype(np.uint32)).to(dev))
    tot = (_i64(client) + _i64(share)) % t
    P = torch.as_tensor(pts).to(dev)
    S = torch.as_tensor(slot_map).to(dev)
    Qd = torch.as_tensor(qrows.astype(np.int32)).to(dev)
    ch = torch.as_tensor(np.asarray(chunks, dtype=np.int64)).to(dev)
    qn2d = torch.as_tensor(qn2).to(dev)
    ar = torch.arange(N, device=dev)
    n_real = 0
    for s in range(0, M, batch):
        e = min(M, s + batch)
        ids = S[ch[s:e, None] * N + ar[None, :]]
        real = ids >= 0
        diff = P[ids.clamp(min=0)].to(torch.int32) - Qd[s:e, None, :]
        dist = (diff * diff).sum(-1).to(torch.int64)
        want = torch.where(real, dist, qn2d[s:e, None])
        assert torch.equal(tot[s:e], want), f"rows {s}..{e - 1}"
        n_real += int(real.sum())
    return n_real


def _select(stage, clustered, srv, sk, out, share, queries, dev):
    """Client step between the phases: decrypt the centre shares and take the
    U closest clusters per query (cleartext stand-in)."""
    ctx = srv.ctx
    C = srv.cdb.n_chunks
    qn2 = ((queries.astype(np.int64) ** 2).sum(axis=1) % ctx.t).astype(np.uint32)
    cl = stage.decrypt_shares(ctx, sk, out.contiguous(),
                              torch.as_tensor(np.repeat(qn2, C)).to(dev)).cpu().numpy()
    sh = share.cpu().numpy()
    sel = []
    for q in range(len(queries)):
        dist = ((cl[q * C:(q + 1) * C].astype(np.int64) + sh[q * C:(q + 1) * C]) % ctx.t)
        sel.append(clustered.select_clusters(dist.reshape(-1), srv.center_slot, U))
    return sel


@pytest.fixture(scope="module")
def cworld():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import clustered, native as nat, stage
    dev = torch.device("cuda")
    w = synthdata.WORKLOADS[4]
    print("\nclustered world: 10M x 96", flush=True)
    cdb = synthdata.gen_clustered(seed=synthdata.SEED_DATA + 4)
    ctx = _digit_ctx(nat, stage, w)
    srv = clustered.ClusteredServer(
        ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
        synthdata.gen_perm(len(cdb.cluster_sizes), synthdata.SEED_PERM + 4),
        synthdata.gen_perm(cdb.stash_size, synthdata.SEED_PERM + 40),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 4),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 40))
    Q = w.Q
    queries = synthdata.gen_queries(w, Q)
    sk, ct = _encrypt(stage, ctx, queries, synthdata.SEED_SK + 4, dev)
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    cout, cshare = srv.center_distances(ct, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    selected = _select(stage, clustered, srv, sk, cout, cshare, queries, dev)
    W = dict(w=w, cdb=cdb, ctx=ctx, srv=srv, Q=Q, queries=queries, sk=sk, ct=ct, qids=qids,
             cout=cout, cshare=cshare, selected=selected, work=srv.work_list(selected),
             nat=nat, stage=stage, clustered=clustered, dev=dev)
    yield W
    W.clear()
    ctx.close()
    torch.cuda.empty_cache()


def test_clustered_full_size_every_query_closed_form(cworld):
    W = cworld
    nat, stage, srv, ctx, dev = W["nat"], W["stage"], W["srv"], W["ctx"], W["dev"]
    Q, queries, cdb = W["Q"], W["queries"], W["cdb"]
    # phase 1: every centre, every query
    Cc = srv.cdb.n_chunks
    n1 = _closed_form(stage, ctx, W["sk"], W["cout"], W["cshare"], np.repeat(queries, Cc, 0),
                      np.tile(np.arange(Cc), Q), srv.center_slot, cdb.centers, dev)
    assert n1 == Q * srv.n_clusters
    # the selection is the U closest centres in the clear
    cen = cdb.centers.astype(np.int64)
    for q in range(Q):
        dq = ((cen - queries[q].astype(np.int64)) ** 2).sum(axis=1)
        sel = np.asarray(W["selected"][q])
        assert len(sel) == U
        assert sorted(dq[sel]) == sorted(np.sort(dq)[:U]), q
    # phase 2: every scanned chunk of every query
    out, share, work = srv.point_distances(W["ct"], W["qids"], W["selected"],
                                           mode=nat.SANNS_MODE_BATCHED)
    torch.cuda.synchronize()
    ctx.device_status()
    assert (work == W["work"]).all()
    n2 = _closed_form(stage, ctx, W["sk"], out, share, queries[work[:, 0]], work[:, 1],
                      srv.layout.slot_point, cdb.points, dev)
    assert set(np.unique(work[:, 0])) == set(range(Q))
    stash = srv.layout.stash_chunks(ctx.N)
    for q in range(Q):
        assert set(stash) <= set(work[work[:, 0] == q, 1]), q
    print(f"checked {n1} centre and {n2} point slots", flush=True)


def _pick_rows(work, stash_first, C):
    """Phase-2 rows: a chunk shared by several queries, a stash chunk, the
    last (padding) chunk, the shortest and the longest per-query lists,
    queries 0 and Q-1, and two more."""
    lens = np.bincount(work[:, 0])
    rows = [0, int(np.nonzero(work[:, 0] == work[-1, 0])[0][0])]
    cl = work[work[:, 1] < stash_first]
    ks, cnt = np.unique(cl[:, 1], return_counts=True)
    shared = ks[cnt >= 2]
    assert len(shared), "no cluster chunk is shared by two queries"
    rows.append(int(np.nonzero(work[:, 1] == shared[len(shared) // 2])[0][0]))
    mid_stash = stash_first + (C - stash_first) // 2
    rows.append(int(np.nonzero(work[:, 1] == mid_stash)[0][0]))
    rows.append(int(np.nonzero(work[:, 1] == C - 1)[0][-1]))
    for q in (int(np.argmin(lens)), int(np.argmax(lens))):
        r = np.nonzero(work[:, 0] == q)[0]
        rows.append(int(r[len(r) // 3]))
    g = np.random.default_rng(len(work))
    rows += [int(x) for x in g.integers(0, len(work), 2)]
    return sorted(set(rows))


def test_clustered_full_size_sampled_rows_against_oracle(cworld):
    W = cworld
    nat, stage, srv, ctx, dev = W["nat"], W["stage"], W["srv"], W["ctx"], W["dev"]
    Q, cdb, work = W["Q"], W["cdb"], W["work"]
    N, L, d = ctx.N, ctx.L, cdb.points.shape[1]
    P = oracle.Params(N, oracle.rns_primes(N, L), oracle.plain_modulus(N, W["w"].t_bits))
    assert P.qs == ctx.qs and P.t == ctx.t
    ct_host = synthdata.gen_uniform_a(P.qs, N, Q * d * 2, 91).reshape(Q, d, 2, L, N)
    ct = torch.as_tensor(ct_host).to(dev)
    qbase = 5000
    qids = torch.as_tensor(np.arange(qbase, qbase + Q, dtype=np.uint64)).to(dev)
    g = np.random.default_rng(92)
    js = sorted(set([0, 1, N - 1] + [int(x) for x in g.integers(0, N, 16)]))

    def check(out, share, rows, pts, slot_map, key):
        for m, (qi, k) in rows:
            print(f"row {m}: query {qi}, chunk {k}", flush=True)
            want_r = oracle.masks(key, qbase + qi, k, P.t, N)
            assert (share[m].cpu().numpy() == want_r).all(), (m, qi, k)
            gk, nrm = oracle.chunk_plaintexts(pts, slot_map, N, k)
            sc, _ = oracle.server_coeffs(P, ct_host[qi], gk, nrm, key, qbase + qi, k, js)
            assert (out[m].cpu().numpy()[:, :, js] == sc).all(), (m, qi, k)

    # phase 1: all-pairs against the centre database
    out1, share1 = srv.center_distances(ct, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    Cc = srv.cdb.n_chunks
    check(out1, share1, [(0, (0, 0)), (Q * Cc - 1, (Q - 1, Cc - 1))], cdb.centers,
          srv.center_slot, srv.key_centers)
    del out1, share1
    # phase 2: per-query chunk lists
    out, share, w2 = srv.point_distances(ct, qids, W["selected"], mode=nat.SANNS_MODE_BATCHED)
    torch.cuda.synchronize()
    ctx.device_status()
    assert (w2 == work).all()
    stash_first = srv.layout.stash_start // N
    rows = _pick_rows(work, stash_first, srv.db.n_chunks)
    assert len(rows) >= 8
    check(out, share, [(m, (int(work[m, 0]), int(work[m, 1]))) for m in rows], cdb.points,
          srv.layout.slot_point, srv.key_points)


def test_serving_full_size_trace(cworld):
    """A Poisson trace over the three resident databases: each request's
    outputs equal the request served alone; every row decrypts to the true
    distances."""
    from paper_1904_02033_amd import serve
    W = cworld
    nat, stage, srv, ctxB, dev = W["nat"], W["stage"], W["srv"], W["ctx"], W["dev"]
    clustered = W["clustered"]
    wA, wB = synthdata.WORKLOADS[2], synthdata.WORKLOADS[3]
    ctxA = _digit_ctx(nat, stage, wA)
    ptsA = synthdata.gen_points(wA, n=100_000, seed=synthdata.SEED_DATA + 5)
    slotA = synthdata.gen_slot_map(len(ptsA), ctxA.N, synthdata.SEED_PERM + 5)
    dbA = stage.encode_db(ctxA, ptsA, slotA)
    ptsB = synthdata.gen_points(wB)
    slotB = synthdata.gen_slot_map(len(ptsB), ctxB.N, synthdata.SEED_PERM + 3)
    dbB = stage.encode_db(ctxB, ptsB, slotB)
    pool = 64
    qA, qB = synthdata.gen_queries(wA, pool), synthdata.gen_queries(wB, pool)
    skA, ctA = _encrypt(stage, ctxA, qA, synthdata.SEED_SK + 5, dev)
    skB, ctB = W["sk"], None
    # the clustered index and database B share ctxB and its client key
    a = synthdata.gen_uniform_a(ctxB.qs, ctxB.N, pool * wB.d, synthdata.SEED_SK + 51)
    e = synthdata.gen_cbd_error(ctxB.N, pool * wB.d, synthdata.SEED_SK + 51)
    ctB = stage.encrypt_query(ctxB, skB, torch.as_tensor(qB.astype(np.int32)).to(dev),
                              torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    del a, e
    dbs = [serve.ResidentDB("A", ctxA, db=dbA, key=synthdata.gen_mask_key(5001)),
           serve.ResidentDB("B", ctxB, db=dbB, key=synthdata.gen_mask_key(5002)),
           serve.ResidentDB("C", ctxB, server=srv, u=U)]

    def select(req, R):
        out, share, _ = req.outputs["centres"]
        return _select(stage, clustered, R.server, skB, out, share, qB[:req.Q], dev)

    arr = synthdata.gen_arrivals(10, 150.0, n_dbs=3, max_q=64, seed=synthdata.SEED_ARR + 5)
    reqs = []
    for r in arr:
        name = "ABC"[r.db]
        reqs.append(serve.Request(r.rid, name, (ctA if name == "A" else ctB)[:r.Q], r.k,
                                  arrival=r.arrival_s))
    print("trace: " + ", ".join(f"{r.db}:{r.Q}" for r in reqs), flush=True)
    server = serve.Server(dbs, hbm_budget=96 << 30, max_inflight=3, max_batch_queries=64,
                          client_select=select, keep_outputs=True)
    done = server.run(reqs, realtime=True)
    assert all(r.done >= 0 and r.error is None for r in done)
    info = {"A": (ctxA, skA, qA, ptsA, slotA, dbA), "B": (ctxB, skB, qB, ptsB, slotB, dbB)}
    for r in done:
        print(f"request {r.rid}: database {r.db}, {r.Q} queries", flush=True)
        qd = torch.as_tensor(r.qids).to(dev)
        if r.db == "C":
            got1, got2 = r.outputs["centres"], r.outputs["points"]
            o1, s1 = srv.center_distances(r.ct, qd, mode=nat.SANNS_MODE_FUSED)
            o2, s2, wk = srv.point_distances(r.ct, qd, r.selected, mode=nat.SANNS_MODE_FUSED)
            torch.cuda.synchronize()
            assert torch.equal(_i64(got1[0]), _i64(o1)) and torch.equal(_i64(got1[1]), _i64(s1))
            assert (got2[2] == wk).all()
            assert torch.equal(_i64(got2[0]), _i64(o2)) and torch.equal(_i64(got2[1]), _i64(s2))
            Cc = srv.cdb.n_chunks
            qs = qB[:r.Q]
            _closed_form(stage, ctxB, skB, got1[0], got1[1], np.repeat(qs, Cc, 0),
                         np.tile(np.arange(Cc), r.Q), srv.center_slot, W["cdb"].centers, dev)
            _closed_form(stage, ctxB, skB, got2[0], got2[1], qs[wk[:, 0]], wk[:, 1],
                         srv.layout.slot_point, W["cdb"].points, dev)
        else:
            ctx, sk, qpool, pts, slot, db = info[r.db]
            R = dbs[0] if r.db == "A" else dbs[1]
            got = r.outputs["scan"]
            o, s = stage.distances(ctx, db, r.ct, R.key, qd)
            torch.cuda.synchronize()
            assert torch.equal(_i64(got[0]), _i64(o)) and torch.equal(_i64(got[1]), _i64(s))
            C = db.n_chunks
            _closed_form(stage, ctx, sk, got[0], got[1], np.repeat(qpool[:r.Q], C, 0),
                         np.tile(np.arange(C), r.Q), slot, pts, dev)
        r.outputs.clear()
        torch.cuda.empty_cache()
    ctxA.close()


def test_clustered_full_size_gathered_phase2(cworld):
    """Phase 2 on per-query gathered chunks plus the resident stash (the
    form that scans only the selected clusters' points): every slot of all
    32 queries decrypts to its distance, and sampled gathered rows equal the
    oracle's on uniform residue inputs."""
    W = cworld
    nat, stage, clustered, ctx, dev = W["nat"], W["stage"], W["clustered"], W["ctx"], W["dev"]
    cdb, Q, queries = W["cdb"], W["Q"], W["queries"]
    gsrv = clustered.ClusteredServer(
        ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
        synthdata.gen_perm(len(cdb.cluster_sizes), synthdata.SEED_PERM + 4),
        synthdata.gen_perm(cdb.stash_size, synthdata.SEED_PERM + 40),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 41), W["srv"].key_centers, gathered=True)
    (co, cs, slot, rq), (so, ss) = gsrv.point_distances_gathered(W["ct"], W["qids"],
                                                                 W["selected"])
    torch.cuda.synchronize()
    ctx.device_status()
    n1 = _closed_form(stage, ctx, W["sk"], co, cs, queries[rq], np.arange(len(rq)), slot,
                      cdb.points, dev)
    assert n1 == W["srv"].requested_pairs(W["selected"]) - Q * cdb.stash_size
    Cs = gsrv.sdb.n_chunks
    n2 = _closed_form(stage, ctx, W["sk"], so, ss, np.repeat(queries, Cs, 0),
                      np.tile(np.arange(Cs), Q), gsrv.stash_slot, cdb.points, dev)
    assert n2 == Q * cdb.stash_size
    del co, cs, so, ss
    # oracle rows on uniform residue inputs
    N, L, d = ctx.N, ctx.L, cdb.points.shape[1]
    P = oracle.Params(N, oracle.rns_primes(N, L), oracle.plain_modulus(N, W["w"].t_bits))
    ct_host = synthdata.gen_uniform_a(P.qs, N, Q * d * 2, 93).reshape(Q, d, 2, L, N)
    qids = torch.as_tensor(np.arange(7000, 7000 + Q, dtype=np.uint64)).to(dev)
    (co, cs, slot, rq), _ = gsrv.point_distances_gathered(torch.as_tensor(ct_host).to(dev), qids,
                                                          W["selected"])
    torch.cuda.synchronize()
    slot = slot.cpu().numpy()
    g = np.random.default_rng(94)
    js = sorted(set([0, N - 1] + [int(x) for x in g.integers(0, N, 16)]))
    last = int(np.nonzero(rq == Q - 1)[0][-1])
    for m in sorted(set([0, last, int(g.integers(0, len(rq)))])):
        qi = int(rq[m])
        want_r = oracle.masks(gsrv.key_points, 7000 + qi, m, P.t, N)
        assert (cs[m].cpu().numpy() == want_r).all(), m
        gk, nrm = oracle.chunk_plaintexts(cdb.points, slot, N, m)
        sc, _ = oracle.server_coeffs(P, ct_host[qi], gk, nrm, gsrv.key_points, 7000 + qi, m, js)
        assert (co[m].cpu().numpy()[:, :, js] == sc).all(), m
