"""The whole batch as one persistent work-queue launch (SANNS_MODE_PERSISTENT):
every built tile shape against the oracle, with query, chunk and coordinate
counts that leave ragged tiles; uneven work lists; graph replays; and the
host-side limits of the mode."""
import numpy as np
import pytest

import oracle
from problem import make_problem, oracle_query_ct, true_distances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# shape id -> (N, L, t_bits) it is built for
SHAPES = {41: (8192, 3, 26), 42: (8192, 3, 26), 43: (8192, 3, 26), 44: (8192, 3, 26),
          51: (4096, 2, 25), 52: (4096, 2, 25), 71: (16384, 3, 26),
          # one 54-bit prime: t small enough that (q mod t) |g|_1 stays below Delta / 2
          61: (2048, 1, 20)}


@pytest.fixture(scope="module")
def stage():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import stage as st
    return st


def _ctx(stage, pb):
    from paper_1904_02033_amd import native as nat
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    p.flags = 0 if pb.P.security_ok() else nat.SANNS_FLAG_INSECURE_TEST
    return stage.Context(params=p)


def _dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _run(stage, pb, mode, work=None, lds=0):
    ctx = _ctx(stage, pb)
    if lds:
        ctx.set_schedule(0, 0, lds)
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    qids = _dev(pb.qids)
    D = stage.Distances(ctx, db, pb.Q, work, mode)
    out, share = D.run(ct, pb.key, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    return ctx, db, sk, ct, qids, D, out.cpu().numpy().copy(), share.cpu().numpy().copy()


def _check_against_oracle(stage, pb, ctx, sk, work, out, share, n_coeffs=24):
    """Server shares in full, ciphertext coefficients at sampled positions
    (first, last and spread ones), and client + server = ||q - p||^2 at every
    slot after decryption."""
    cts = {}
    N = pb.N
    js = sorted(set([0, 1, N - 1] + list(np.random.default_rng(N).integers(0, N, n_coeffs))))
    for m, (qi, k) in enumerate(work):
        assert (share[m] == oracle.masks(pb.key, int(pb.qids[qi]), k, pb.P.t, N)).all(), m
        if qi not in cts:
            cts[qi] = oracle_query_ct(pb, qi)
        g, nrm = oracle.chunk_plaintexts(pb.pts, pb.slot, N, k)
        sc, sr = oracle.server_coeffs(pb.P, cts[qi], g, nrm, pb.key, int(pb.qids[qi]), k, js)
        assert (out[m][:, :, js] == sc).all(), m
        assert (share[m][js] == sr).all(), m
    owner = np.array([w[0] for w in work])
    client = stage.decrypt_shares(ctx, sk, _dev(out), _dev(pb.qnorm2()[owner])).cpu().numpy()
    for m, (qi, k) in enumerate(work):
        dist = true_distances(pb, qi, k)
        tot = (client[m].astype(np.int64) + share[m].astype(np.int64)) % pb.P.t
        real = dist >= 0
        assert (tot[real] == dist[real]).all(), (m, qi, k)


@pytest.mark.parametrize("shape", sorted(SHAPES))
def test_persistent_shape_matches_oracle_and_fused(stage, shape):
    from paper_1904_02033_amd import native as nat
    N, L, tb = SHAPES[shape]
    # 5 queries, 3 chunks (the last one partly padding), d = 7: ragged against
    # every tile of queries, chunks and staged coordinates
    pb = make_problem(N, L, tb, 2 * N + 77, 7, 5, "i8" if shape % 2 else "u8", seed=shape)
    ctx, db, sk, ct, qids, D, out, share = _run(stage, pb, nat.SANNS_MODE_PERSISTENT,
                                                lds=shape)
    work = [(q, k) for q in range(pb.Q) for k in range(pb.C)]
    _check_against_oracle(stage, pb, ctx, sk, work, out, share)
    F = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_FUSED)
    fo, fs = F.run(ct, pb.key, qids)
    torch.cuda.synchronize()
    assert (fo.cpu().numpy() == out).all() and (fs.cpu().numpy() == share).all()


@pytest.mark.parametrize("N,L,tb", [(4096, 2, 25), (8192, 3, 26)])
def test_persistent_uneven_work_list(stage, N, L, tb):
    """Per-query chunk lists of different lengths, repeated and reordered
    (register tiles from a host-built table inside the persistent launch)."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(N, L, tb, 4 * N + 5, 6, 4, "u8", seed=N + 1)
    g = np.random.default_rng(N)
    work = []
    for qi in range(pb.Q):
        ks = g.choice(pb.C, size=int(g.integers(1, pb.C + 1)), replace=False)
        work += [(qi, int(k)) for k in ks]
    work = [work[i] for i in g.permutation(len(work))]
    warr = np.array(work, dtype=np.uint32)
    ctx, db, sk, ct, qids, D, out, share = _run(stage, pb, nat.SANNS_MODE_PERSISTENT, warr)
    _check_against_oracle(stage, pb, ctx, sk, work, out, share, n_coeffs=8)
    F = stage.Distances(ctx, db, pb.Q, warr, nat.SANNS_MODE_FUSED)
    fo, fs = F.run(ct, pb.key, qids)
    torch.cuda.synchronize()
    assert (fo.cpu().numpy() == out).all() and (fs.cpu().numpy() == share).all()


def test_persistent_graph_replays_pick_up_new_inputs(stage):
    """The captured launch (counter reset included) replays correctly, with
    eager work and synchronisation between replays."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(4096, 2, 25, 3 * 4096 + 11, 5, 3, "u8", seed=31)
    ctx, db, sk, ct, qids, D, out1, share1 = _run(stage, pb, nat.SANNS_MODE_FUSED)
    P = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_PERSISTENT)
    for rep in range(4):
        if rep == 2:
            # new query order and ids: the replay must read the new contents
            ct.copy_(ct.flip(0).contiguous())
            qids.copy_(qids.flip(0).contiguous())
            F = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_FUSED)
            fo, fs = F.run(ct, pb.key, qids)
            torch.cuda.synchronize()
            out1, share1 = fo.cpu().numpy().copy(), fs.cpu().numpy().copy()
        o, s = P.run(ct, pb.key, qids)
        torch.zeros(1 << 20, device="cuda").add_(1.0)  # unrelated eager work
        torch.cuda.synchronize()
        ctx.device_status()
        assert (o.cpu().numpy() == out1).all() and (s.cpu().numpy() == share1).all(), rep


def test_persistent_limits_are_host_errors(stage):
    from paper_1904_02033_amd import native as nat
    small = make_problem(1024, 1, 20, 100, 3, 2, "u8", seed=3)
    ctx = _ctx(stage, small)
    db = stage.encode_db(ctx, small.pts, small.slot)
    D = stage.Distances(ctx, db, 2, None, nat.SANNS_MODE_PERSISTENT)
    ct = torch.zeros((2, 3, 2, 1, 1024), dtype=torch.uint64, device="cuda")
    q = torch.zeros(2, dtype=torch.uint64, device="cuda")
    with pytest.raises(nat.SannsError) as ei:
        D.run(ct, small.key, q)
    assert ei.value.status == nat.SANNS_E_INVALID
    wide = make_problem(4096, 2, 26, 40, 300, 1, "u8", seed=4)
    ctx = _ctx(stage, wide)
    db = stage.encode_db(ctx, wide.pts, wide.slot)
    D = stage.Distances(ctx, db, 1, None, nat.SANNS_MODE_PERSISTENT)
    ct = torch.zeros((1, 300, 2, 2, 4096), dtype=torch.uint64, device="cuda")
    with pytest.raises(nat.SannsError) as ei:
        D.run(ct, wide.key, q[:1])
    assert ei.value.status == nat.SANNS_E_INVALID
    with pytest.raises(nat.SannsError):
        ctx.set_schedule(0, 0, 41)  # a shape built for N = 8192
