"""Distances on chunks gathered per call (sanns_distances_gathered) through
the C ABI: retrieved points of each query packed into fresh chunks and
encoded on the fly (clustering-based protocol, steps 6-7), and the same on
the server's additive shares of secret-shared points (Section 4.2, last
paragraph).  Every output row against the oracle, every slot against the
cleartext distances, the host and device limits, and the clustered form's
gathered phase 2 against its resident phase 2."""
import numpy as np
import pytest

import oracle
import synthdata
from problem import make_problem, oracle_query_ct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import clustered, native as nat, stage
    return nat, stage, clustered


def _dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _ctx(nat, stage, pb):
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    if not pb.P.security_ok():
        p.flags |= nat.SANNS_FLAG_INSECURE_TEST
    return stage.Context(params=p)


def _plan(N, lists):
    slots, rows = [], []
    for q, idx in enumerate(lists):
        m = max(1, (len(idx) + N - 1) // N)
        blk = np.full(m * N, -1, dtype=np.int64)
        blk[:len(idx)] = idx
        slots.append(blk)
        rows += [q] * m
    return np.concatenate(slots), np.array(rows, dtype=np.uint32)


def _run(nat, stage, pb, share_mode, lists, seed, tail_n=0):
    ctx = _ctx(nat, stage, pb)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    slot, rq = _plan(pb.N, lists)
    tail, tslot, Ct = None, None, 0
    if tail_n:
        # a resident tail database over the first tail_n points (the stash)
        tslot = synthdata.gen_slot_map(tail_n, pb.N, seed + 11)
        tail = stage.encode_db(ctx, pb.pts, tslot)
        Ct = tail.n_chunks
    g = np.random.default_rng(seed)
    n, d = pb.pts.shape
    pts64 = pb.pts.astype(np.int64)
    if share_mode:
        pc = g.integers(0, pb.P.t, (n, d)).astype(np.int64)
        psh = ((pts64 - pc) % pb.P.t).astype(np.uint32)
        nc = g.integers(0, pb.P.t, n).astype(np.int64)
        nsh = (((pts64 ** 2).sum(axis=1) - nc) % pb.P.t).astype(np.uint32)
        out, share = stage.gathered_distances(ctx, _dev(psh.view(np.int32)), slot, rq, ct,
                                              pb.key, _dev(pb.qids), norm_shares=_dev(nsh))
    else:
        out, share = stage.gathered_distances(ctx, _dev(pb.pts), slot, rq, ct, pb.key,
                                              _dev(pb.qids), tail=tail)
    torch.cuda.synchronize()
    ctx.device_status()
    M = len(rq)
    assert out.shape[0] == M + pb.Q * Ct
    if Ct:
        # tail rows M + q Ct + k: (query q, tail chunk k), mask chunk word M + k
        tout, tshare = out[M:].cpu().numpy(), share[M:].cpu().numpy()
        for q in range(pb.Q):
            ctq = oracle_query_ct(pb, q)
            for k in range(Ct):
                gk, nrm = oracle.chunk_plaintexts(pb.pts, tslot, pb.N, k)
                w_ct, w_r = oracle.server_chunk(pb.P, ctq, gk, nrm, pb.key, int(pb.qids[q]),
                                                M + k)
                assert (tout[q * Ct + k] == w_ct).all(), (q, k)
                assert (tshare[q * Ct + k] == w_r).all(), (q, k)
        out, share = out[:M], share[:M]
    out_h, share_h = out.cpu().numpy(), share.cpu().numpy()
    cts = {}
    for m in range(M):
        qi = int(rq[m])
        if qi not in cts:
            cts[qi] = oracle_query_ct(pb, qi)
        if share_mode:
            gk, nrm = oracle.chunk_plaintexts_shares(psh, nsh, slot, pb.N, m, pb.P.t)
        else:
            gk, nrm = oracle.chunk_plaintexts(pb.pts, slot, pb.N, m)
        w_ct, w_r = oracle.server_chunk(pb.P, cts[qi], gk, nrm, pb.key, int(pb.qids[qi]), m)
        assert (out_h[m] == w_ct).all(), m
        assert (share_h[m] == w_r).all(), m
    # every slot: client + server = ||q - p||^2
    client = stage.decrypt_shares(ctx, sk, out, _dev(pb.qnorm2()[rq])).cpu().numpy()
    for m in range(M):
        qi = int(rq[m])
        ids = slot[m * pb.N:(m + 1) * pb.N]
        real = ids >= 0
        c = client[m].astype(np.int64)
        if share_mode:
            q64 = pb.queries[qi].astype(np.int64)
            c[real] += -2 * (pc[ids[real]] @ q64) + nc[ids[real]]
        tot = (c + share_h[m]) % pb.P.t
        want = ((pts64[ids[real]] - pb.queries[qi].astype(np.int64)) ** 2).sum(axis=1)
        assert (tot[real] == want).all(), m
    ctx.close()
    return M


@pytest.mark.parametrize("share_mode", [False, True], ids=["points", "shares"])
@pytest.mark.parametrize("N,L,tb,dt", [(4096, 2, 25, "u8"), (8192, 3, 26, "i8"),
                                       (1024, 2, 21, "u8")])
def test_gathered_rows_match_oracle(mods, share_mode, N, L, tb, dt):
    nat, stage, _ = mods
    n, d = 3 * N + 50, 12
    pb = make_problem(N, L, tb, n, d, 3, dt, seed=N + 7 * share_mode + 1)
    g = np.random.default_rng(N)
    lists = [g.choice(n, size=N + 37, replace=False), g.choice(n, size=5, replace=False),
             g.permutation(n)[:2 * N]]
    M = _run(nat, stage, pb, share_mode, lists, seed=N + 3,
             tail_n=0 if share_mode else N + 100)
    assert M == 2 + 1 + 2


def test_gathered_limits(mods):
    nat, stage, _ = mods
    pb = make_problem(4096, 2, 25, 100, 4, 2, "u8", seed=71)
    ctx = _ctx(nat, stage, pb)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    slot, rq = _plan(4096, [np.arange(10), np.arange(20)])
    with pytest.raises(nat.SannsError) as ei:
        stage.gathered_distances(ctx, _dev(pb.pts), slot, np.array([0, 2], np.uint32), ct,
                                 pb.key, _dev(pb.qids))
    assert ei.value.status == nat.SANNS_E_RANGE
    with pytest.raises(nat.SannsError) as ei:
        stage.gathered_distances(ctx, _dev(pb.pts.astype(np.int32)), slot, rq, ct, pb.key,
                                 _dev(pb.qids))
    assert ei.value.status == nat.SANNS_E_INVALID      # shares need their norm shares
    bad = np.zeros((100, 4), dtype=np.uint32)
    bad[3, 1] = pb.P.t                                  # a share >= t
    stage.gathered_distances(ctx, _dev(bad.view(np.int32)), slot, rq, ct, pb.key,
                             _dev(pb.qids), norm_shares=_dev(np.zeros(100, np.uint32)))
    with pytest.raises(nat.SannsError) as ei:
        ctx.device_status()
    assert ei.value.status == nat.SANNS_E_RANGE
    slot2 = slot.copy()
    slot2[7] = 100                                      # past the last point
    stage.gathered_distances(ctx, _dev(pb.pts), slot2, rq, ct, pb.key, _dev(pb.qids))
    with pytest.raises(nat.SannsError) as ei:
        ctx.device_status()
    assert ei.value.status == nat.SANNS_E_RANGE
    ctx.device_status()
    ctx.close()


def test_clustered_gathered_phase2_equals_resident(mods):
    """The clustered index in both forms: the gathered phase 2 reconstructs
    the same distances as the resident one for every selected point and the
    stash."""
    nat, stage, clustered = mods
    N = 4096
    P = oracle.Params(N, oracle.rns_primes(N, 2), oracle.plain_modulus(N, 26))
    p = nat.sanns_params()
    p.N, p.L, p.t = N, 2, P.t
    for l, q in enumerate(P.qs):
        p.q[l] = q
    ctx = stage.Context(params=p)
    cdb = synthdata.gen_clustered(n_clusters=60, total_clustered=15000, stash=1300, d=24,
                                  seed=8)
    args = (ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
            synthdata.gen_perm(60, 3), synthdata.gen_perm(1300, 4),
            synthdata.gen_mask_key(10), synthdata.gen_mask_key(11))
    res = clustered.ClusteredServer(*args)
    gat = clustered.ClusteredServer(*(args[:7] + (synthdata.gen_mask_key(12), args[8])),
                                    gathered=True)
    Q = 3
    g = np.random.default_rng(9)
    queries = g.integers(-127, 128, (Q, 24)).astype(np.int8)
    sk = _dev(synthdata.gen_secret(N, 13))
    a = synthdata.gen_uniform_a(P.qs, N, Q * 24, 14)
    e = synthdata.gen_cbd_error(N, Q * 24, 14)
    ct = stage.encrypt_query(ctx, sk, _dev(queries, torch.int32), _dev(a), _dev(e))
    qids = _dev(np.arange(Q, dtype=np.uint64))
    selected = [g.choice(60, size=7, replace=False) for _ in range(Q)]
    qn2 = ((queries.astype(np.int64) ** 2).sum(axis=1) % P.t).astype(np.uint32)

    def dist_of(out, share, owner):
        cl = stage.decrypt_shares(ctx, sk, out.contiguous(), _dev(qn2[owner])).cpu().numpy()
        return (cl.astype(np.int64) + share.cpu().numpy()) % P.t

    out, share, work = res.point_distances(ct, qids, selected)
    dres = dist_of(out, share, work[:, 0])
    (co, cs, slot, rq), (so, ss) = gat.point_distances_gathered(ct, qids, selected)
    slot = slot.cpu().numpy()
    hs, hq = gat.gather_plan(selected)  # the host plan gives the same map
    assert (hs == slot).all() and (hq == rq).all()
    dgc = dist_of(co, cs, rq)
    dgs = dist_of(so, ss, np.repeat(np.arange(Q), gat.sdb.n_chunks))
    torch.cuda.synchronize()
    ctx.device_status()
    lay = res.layout
    for q in range(Q):
        # resident: distance of every slot of this query's rows, by point id
        want = {}
        for m in np.nonzero(work[:, 0] == q)[0]:
            ids = lay.slot_point[work[m, 1] * N:(work[m, 1] + 1) * N]
            for j, i in enumerate(ids):
                if i >= 0:
                    want[int(i)] = int(dres[m, j])
        got = {}
        for m in np.nonzero(rq == q)[0]:
            ids = slot[m * N:(m + 1) * N]
            for j, i in enumerate(ids):
                if i >= 0:
                    got[int(i)] = int(dgc[m, j])
        Cs = gat.sdb.n_chunks
        for k in range(Cs):
            ids = gat.stash_slot[k * N:(k + 1) * N]
            for j, i in enumerate(ids):
                if i >= 0:
                    got[int(i)] = int(dgs[q * Cs + k, j])
        sel_pts = set(int(i) for c in selected[q]
                      for i in range(lay.cluster_start[c], lay.cluster_end[c]))
        stash_pts = set(int(i) for i in lay.slot_point[lay.stash_start:lay.stash_end])
        assert set(got) == sel_pts | stash_pts
        for i in got:
            assert got[i] == want[i], (q, i)
            assert got[i] == int(((cdb.points[i].astype(np.int64) - queries[q]) ** 2).sum())
    ctx.close()
