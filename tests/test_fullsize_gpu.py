"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (64 queries against a resident 1M-point database, N = 8192,
L = 3; batched graph and persistent launch; the clustered 10M form).

At these sizes the oracle cannot produce every output, so each test checks
  * bit-exact server shares of sampled output rows, in full, against the
    oracle's ChaCha20 masks;
  * bit-exact ciphertext coefficients at sampled (output, position) pairs
    against the oracle's one-coefficient-at-a-time products, on synthetic
    residue inputs fed to both sides;
  * the property that holds at any size: after decryption, client + server
    shares equal the cleartext squared distance at every slot of every
    output (the reference distances come from an exact float64 matmul:
    every inner product is below 2^53).
"""
import numpy as np
import pytest

import oracle
import synthdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _i64(x):
    """uint32 / uint64 device tensor -> int64 values (bit views; no unsigned
    arithmetic on the device)."""
    if x.dtype == torch.uint32:
        return x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return x.view(torch.int64)


def _world(cid):
    from paper_1904_02033_amd import stage
    w = dataclass_for(cid)
    pts = synthdata.gen_points(w)
    queries = synthdata.gen_queries(w, 64)
    ctx = stage.Context(w.N, w.L, w.t_bits)
    slot = stage.linear_slot_map(len(pts), ctx.N,
                                 synthdata.gen_perm(len(pts), synthdata.SEED_PERM + w.cid))
    db = stage.encode_db(ctx, pts, slot)
    return w, pts, queries, ctx, slot, db


def dataclass_for(cid):
    return synthdata.BATCHED_1M128 if cid == 2 else synthdata.WORKLOADS[cid]


def _true_dist_slots(pts, queries, slot, dev):
    """[Q][C N] int64 squared distances per slot (-1 for padding)."""
    p = torch.as_tensor(pts.astype(np.float64)).to(dev)
    q = torch.as_tensor(queries.astype(np.float64)).to(dev)
    dots = q @ p.T                                        # exact: < 2^53
    d2 = ((q * q).sum(1, keepdim=True) + (p * p).sum(1)[None, :] - 2.0 * dots)
    d2 = d2.round().to(torch.int64)
    sl = torch.as_tensor(slot).to(dev)
    out = torch.full((len(queries), len(slot)), -1, dtype=torch.int64, device=dev)
    real = sl >= 0
    out[:, real] = d2[:, sl[real]]
    return out


@pytest.mark.parametrize("cid", [2, 3])
def test_full_size_batch_shares_are_distances(cid):
    """64 encrypted queries against the 1M-point database: batched graph and
    persistent launch agree bit for bit, and decrypt to the true distances at
    every slot."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import native as nat, stage
    dev = torch.device("cuda")
    w, pts, queries, ctx, slot, db = _world(cid)
    Q, d, C, N, L, t = 64, pts.shape[1], db.n_chunks, ctx.N, ctx.L, ctx.t
    sk = torch.as_tensor(synthdata.gen_secret(N, synthdata.SEED_SK + cid)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, N, Q * d, synthdata.SEED_ENC + cid)
    e = synthdata.gen_cbd_error(N, Q * d, synthdata.SEED_ENC + cid)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    del a, e
    key = synthdata.gen_mask_key(synthdata.SEED_MASK + cid)
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    B = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED)
    bo, bs = B.run(ct, key, qids)
    P = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_PERSISTENT)
    po, ps = P.run(ct, key, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    assert torch.equal(_i64(bo), _i64(po)) and torch.equal(_i64(bs), _i64(ps))
    del P, po, ps
    qn2 = ((queries.astype(np.int64) ** 2).sum(axis=1) % t).astype(np.uint32)
    client = stage.decrypt_shares(ctx, sk, bo, torch.as_tensor(np.repeat(qn2, C)).to(dev))
    tot = (_i64(client) + _i64(bs)) % t                   # [Q C][N]
    want = _true_dist_slots(pts, queries, slot, dev)      # [Q][C N]
    tot = tot.view(Q, C * N)
    real = want >= 0
    assert torch.equal(tot[real], want[real])
    # padding slots carry ||q||^2 (a zero point)
    pad = ~real
    assert torch.equal(tot[pad], torch.as_tensor(qn2.astype(np.int64)).to(dev)[:, None]
                       .expand(Q, C * N)[pad])


def test_full_size_batch_sampled_against_oracle():
    """Synthetic residue inputs (both sides get the same bytes): server
    shares of sampled rows in full and ciphertext coefficients at sampled
    positions, for the batched graph at 1M x 128, 64 queries."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import native as nat, stage
    dev = torch.device("cuda")
    w, pts, queries, ctx, slot, db = _world(2)
    Q, d, C, N, L = 64, pts.shape[1], db.n_chunks, ctx.N, ctx.L
    P = oracle.Params(N, oracle.rns_primes(N, L), ctx.t)
    ct_host = synthdata.gen_uniform_a(P.qs, N, Q * d * 2, 77).reshape(Q, d, 2, L, N)
    ct = torch.as_tensor(ct_host).to(dev)
    key = synthdata.gen_mask_key(78)
    qids = torch.as_tensor(np.arange(1000, 1000 + Q, dtype=np.uint64)).to(dev)
    B = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED)
    out, share = B.run(ct, key, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    g = np.random.default_rng(79)
    rows = sorted(set([0, Q * C - 1] + list(g.integers(0, Q * C, 10))))
    js = sorted(set([0, N - 1] + list(g.integers(0, N, 4))))
    for m in rows:
        qi, k = divmod(m, C)
        want_r = oracle.masks(key, 1000 + qi, k, P.t, N)
        assert (share[m].cpu().numpy() == want_r).all(), m
        gk, nrm = oracle.chunk_plaintexts(pts, slot, N, k)
        sc, sr = oracle.server_coeffs(P, ct_host[qi], gk, nrm, key, 1000 + qi, k, js)
        got = out[m].cpu().numpy()[:, :, js]
        assert (got == sc).all(), m


def test_full_size_clustered_shares_are_distances():
    """The clustered 10M x 96 form with the benchmark's 32 queries x 64
    clusters: phase-2 outputs of two queries decrypt to the true distances at
    every slot of every chunk they scanned."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import clustered, native as nat, stage
    dev = torch.device("cuda")
    w = synthdata.WORKLOADS[4]
    cdb = synthdata.gen_clustered(seed=synthdata.SEED_DATA + 4)
    ctx = stage.Context(w.N, w.L, w.t_bits)
    srv = clustered.ClusteredServer(
        ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
        synthdata.gen_perm(len(cdb.cluster_sizes), synthdata.SEED_PERM + 4),
        synthdata.gen_perm(cdb.stash_size, synthdata.SEED_PERM + 40),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 4),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 40))
    Q, u, t, N = w.Q, 64, ctx.t, ctx.N
    queries = synthdata.gen_queries(w, Q)
    sk = torch.as_tensor(synthdata.gen_secret(N, synthdata.SEED_SK + 4)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, N, Q * w.d, synthdata.SEED_SK + 5)
    e = synthdata.gen_cbd_error(N, Q * w.d, synthdata.SEED_SK + 5)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    qn2 = ((queries.astype(np.int64) ** 2).sum(axis=1) % t).astype(np.uint32)
    cout, cshare = srv.center_distances(ct, qids)
    Cc = srv.cdb.n_chunks
    cl = stage.decrypt_shares(ctx, sk, cout, torch.as_tensor(np.repeat(qn2, Cc)).to(dev))
    cl, cs = cl.cpu().numpy(), cshare.cpu().numpy()
    selected = [clustered.select_clusters(
        ((cl[q * Cc:(q + 1) * Cc].astype(np.int64) + cs[q * Cc:(q + 1) * Cc]) % t).reshape(-1),
        srv.center_slot, u) for q in range(Q)]
    out, share, work = srv.point_distances(ct, qids, selected, mode=nat.SANNS_MODE_BATCHED)
    client = stage.decrypt_shares(ctx, sk, out, torch.as_tensor(qn2[work[:, 0]]).to(dev))
    tot = ((client.cpu().numpy().astype(np.int64) + share.cpu().numpy()) % t)
    for q in (0, Q - 1):
        rows = np.nonzero(work[:, 0] == q)[0]
        assert len(rows) >= 13  # at least the stash chunks
        for m in rows:
            ids = srv.layout.slot_point[work[m, 1] * N:(work[m, 1] + 1) * N]
            real = ids >= 0
            want = ((cdb.points[ids[real]].astype(np.int64) - queries[q]) ** 2).sum(axis=1)
            assert (tot[m][real] == want).all(), (q, m)
