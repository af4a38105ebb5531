"""Continuous-batching loop: every request's outputs are bit-identical to the
same request served alone, shares reconstruct the true distances, admission
respects the HBM budget, and an oversized request is refused."""
import numpy as np
import pytest

import oracle
import synthdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(stage, nat, N, L, tb):
    P = oracle.Params(N, oracle.rns_primes(N, L), oracle.plain_modulus(N, tb))
    p = nat.sanns_params()
    p.N, p.L, p.t = N, L, P.t
    for l, q in enumerate(P.qs):
        p.q[l] = q
    return stage.Context(params=p)


@pytest.fixture(scope="module")
def world():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import clustered, native as nat, serve, stage
    N = 4096
    ctxA = _ctx(stage, nat, N, 2, 25)
    ctxB = _ctx(stage, nat, N, 2, 26)
    g = np.random.default_rng(5)
    ptsA = g.integers(0, 256, (6000, 16)).astype(np.uint8)
    ptsB = g.integers(-127, 128, (9000, 24)).astype(np.int8)
    dbA = stage.encode_db(ctxA, ptsA, stage.linear_slot_map(6000, N, synthdata.gen_perm(6000, 1)))
    dbB = stage.encode_db(ctxB, ptsB, stage.linear_slot_map(9000, N, synthdata.gen_perm(9000, 2)))
    cdb = synthdata.gen_clustered(n_clusters=40, total_clustered=12000, stash=900, d=24, seed=6)
    srv = clustered.ClusteredServer(ctxB, cdb.points, cdb.cluster_sizes, cdb.centers,
                                    cdb.stash_size, synthdata.gen_perm(40, 3),
                                    synthdata.gen_perm(900, 4), synthdata.gen_mask_key(10),
                                    synthdata.gen_mask_key(11))
    dbs = [serve.ResidentDB("A", ctxA, db=dbA, key=synthdata.gen_mask_key(12)),
           serve.ResidentDB("B", ctxB, db=dbB, key=synthdata.gen_mask_key(13)),
           serve.ResidentDB("C", ctxB, server=srv, u=5)]
    skA = torch.as_tensor(synthdata.gen_secret(N, 20)).cuda()
    skB = torch.as_tensor(synthdata.gen_secret(N, 21)).cuda()
    return dict(nat=nat, serve=serve, stage=stage, clustered=clustered, ctx={"A": ctxA,
                "B": ctxB, "C": ctxB}, pts={"A": ptsA, "B": ptsB, "C": cdb.points},
                dbs=dbs, sk={"A": skA, "B": skB, "C": skB}, cdb=cdb, srv=srv)


def _requests(W, n_req, seed):
    serve = W["serve"]
    g = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        name = "ABC"[int(g.integers(0, 3))]
        ctx = W["ctx"][name]
        d = W["pts"][name].shape[1]
        Q = int(g.integers(1, 5))
        if name == "A":
            qs = g.integers(0, 256, (Q, d))
        else:
            qs = g.integers(-127, 128, (Q, d))
        a = synthdata.gen_uniform_a(ctx.qs, ctx.N, Q * d, 100 + r)
        e = synthdata.gen_cbd_error(ctx.N, Q * d, 100 + r)
        ct = W["stage"].encrypt_query(ctx, W["sk"][name], torch.as_tensor(qs.astype(np.int32)).cuda(),
                                      torch.as_tensor(a).cuda(), torch.as_tensor(e).cuda())
        req = serve.Request(r, name, ct, 10, arrival=float(g.uniform(0, 0.02)))
        req.queries = qs
        reqs.append(req)
    torch.cuda.synchronize()
    return reqs


def _client_select(W):
    stage, clustered = W["stage"], W["clustered"]

    def select(req, R):
        out, share, _ = req.outputs["centres"]
        ctx = R.ctx
        C = R.server.cdb.n_chunks
        qn2 = ((req.queries.astype(np.int64) ** 2).sum(axis=1) % ctx.t).astype(np.uint32)
        cl = stage.decrypt_shares(ctx, W["sk"]["C"], out.contiguous(),
                                  torch.as_tensor(np.repeat(qn2, C)).cuda()).cpu().numpy()
        sh = share.cpu().numpy()
        sel = []
        for q in range(req.Q):
            dist = ((cl[q * C:(q + 1) * C].astype(np.int64) + sh[q * C:(q + 1) * C])
                    % ctx.t).reshape(-1)
            sel.append(clustered.select_clusters(dist, R.server.center_slot, R.u))
        return sel
    return select


@pytest.mark.parametrize("realtime", [True, False], ids=["arrivals", "all-at-once"])
def test_mix_equals_alone_and_shares_are_distances(world, realtime):
    """With real-time arrivals (admitted as they come) and with every request
    queued at once (so that launches must pack several requests): each
    request's outputs equal the request served alone."""
    W = world
    serve, stage, nat = W["serve"], W["stage"], W["nat"]
    reqs = _requests(W, 14, seed=1)
    server = serve.Server(W["dbs"], hbm_budget=1 << 30, max_inflight=3, max_batch_queries=5,
                          client_select=_client_select(W))
    done = server.run(reqs, realtime=realtime)
    assert all(r.done >= 0 for r in done)
    if not realtime:
        assert server.launches < sum(1 + (r.db == "C") for r in reqs), "nothing was batched"
    for r in done:
        R = next(d for d in W["dbs"] if d.name == r.db)
        ctx = W["ctx"][r.db]
        qd = torch.as_tensor(r.qids).cuda()
        if r.db == "C":
            out, share = R.server.center_distances(r.ct, qd, mode=nat.SANNS_MODE_FUSED)
            got = r.outputs["centres"]
            assert (got[0].cpu().numpy() == out.cpu().numpy()).all()
            assert (got[1].cpu().numpy() == share.cpu().numpy()).all()
            out, share, work = R.server.point_distances(r.ct, qd, r.selected,
                                                        mode=nat.SANNS_MODE_FUSED)
            got = r.outputs["points"]
            assert (got[2] == work).all()
        else:
            out, share = stage.distances(ctx, R.db, r.ct, R.key, qd)
            got = r.outputs["scan"]
            work = None
        torch.cuda.synchronize()
        assert (got[0].cpu().numpy() == out.cpu().numpy()).all(), r.rid
        assert (got[1].cpu().numpy() == share.cpu().numpy()).all(), r.rid
        # the shares reconstruct ||q - p||^2 for the first output of each query
        qn2 = ((r.queries.astype(np.int64) ** 2).sum(axis=1) % ctx.t).astype(np.uint32)
        if work is None:
            C = R.db.n_chunks
            owner = np.repeat(np.arange(r.Q), C)
            chunk = np.tile(np.arange(C), r.Q)
            slot_map, pts = R.db.slot_point.cpu().numpy(), W["pts"][r.db]
        else:
            owner, chunk = work[:, 0], work[:, 1]
            slot_map, pts = R.server.layout.slot_point, W["pts"]["C"]
        cl = stage.decrypt_shares(ctx, W["sk"][r.db], got[0].contiguous(),
                                  torch.as_tensor(qn2[owner]).cuda()).cpu().numpy()
        sh = got[1].cpu().numpy()
        for m in range(min(3, len(owner))):
            ids = slot_map[chunk[m] * ctx.N:(chunk[m] + 1) * ctx.N]
            real = ids >= 0
            tot = (cl[m].astype(np.int64) + sh[m]) % ctx.t
            assert (tot[real] == oracle.sqdist(r.queries[owner[m]], pts[ids[real]])).all()


def test_admission_budget_and_rejection(world):
    W = world
    serve = W["serve"]
    reqs = _requests(W, 8, seed=2)
    one = max(serve.Server(W["dbs"], 1 << 40)._footprint(
        r.db, "centres" if r.db == "C" else "scan", r.Q,
        r.Q * (W["srv"].cdb.n_chunks if r.db == "C" else
               next(d for d in W["dbs"] if d.name == r.db).db.n_chunks)) for r in reqs)
    budget = int(one * 1.6)
    for keep in (False, True):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        server = serve.Server(W["dbs"], hbm_budget=budget, max_inflight=3,
                              max_batch_queries=8, client_select=_client_select(W),
                              keep_outputs=keep)
        done = server.run(reqs, realtime=False)
        assert all(r.done >= 0 and r.error is None for r in done)
        assert server.peak_used <= budget
        if not keep:
            # everything the loop allocated stays within the budget; the
            # client's decryptions inside client_select (a few KiB) and the
            # allocator's rounding are the slack
            peak = torch.cuda.max_memory_allocated() - base
            assert peak <= budget + (4 << 20), (peak, budget)
        del server, done
    tiny = serve.Server(W["dbs"], hbm_budget=1 << 20)
    with pytest.raises(serve.AdmissionError):
        tiny.submit(reqs[0])


def test_query_ids_are_never_reused(world):
    """Masks are drawn from (database key, query id, chunk): the loop assigns
    every query's id from the database's own counter, so two requests, or
    two runs of the loop over the same database, never share an id."""
    W = world
    serve = W["serve"]
    reqs = _requests(W, 6, seed=3)
    for r in reqs:
        r.qids = np.zeros(r.Q, dtype=np.uint64)  # a client's choice is ignored
    seen = {}
    for run in range(2):
        server = serve.Server(W["dbs"], hbm_budget=1 << 34, max_inflight=2,
                              max_batch_queries=8, client_select=_client_select(W),
                              keep_outputs=False)
        for r in reqs:
            r.outputs.clear()
        done = server.run(reqs, realtime=False)
        for r in done:
            assert len(r.qids) == r.Q
            for q in r.qids:
                k = (r.db if r.db != "C" else "C", int(q))
                assert k not in seen, f"query id {int(q)} reused under database {r.db}"
                seen[k] = r.rid
