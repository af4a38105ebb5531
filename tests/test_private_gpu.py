"""The circuit-private form (sanns_distances_cp: re-randomisation under the
client's public key plus noise flooding, Section 2.3) through the C ABI
against the oracle: every output ciphertext bit for bit at small rings, in
the fused and graph forms, with the vector and matrix-core schedules and
with work lists; the shares unchanged and still reconstructing the
distances; the public key helper against the oracle's; host-side limits."""
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
    from paper_1904_02033_amd import native as nat, stage
    return nat, stage


def _dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _setup(nat, stage, pb, digits=False):
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    if not pb.P.security_ok():
        p.flags |= nat.SANNS_FLAG_INSECURE_TEST
    if digits:
        p.flags |= nat.SANNS_FLAG_DIGIT_DB
    ctx = stage.Context(params=p)
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    return ctx, db, sk, ct, _dev(pb.qids)


def _public_keys(stage, ctx, pb, sk, seed):
    """Q public keys (one per query, as separate clients would send)."""
    pks = [oracle.sample_public_key(pb.P, pb.sk, seed + q) for q in range(pb.Q)]
    got = [stage.public_key(ctx, sk, seed + q) for q in range(pb.Q)]
    torch.cuda.synchronize()
    for q in range(pb.Q):
        assert (got[q].cpu().numpy() == pks[q]).all(), q
    return np.stack(pks), torch.stack(got).contiguous()


def _oracle_rows(pb, pks, rows, b, cts):
    out = {}
    for m, (qi, k) in rows:
        if qi not in cts:
            cts[qi] = oracle_query_ct(pb, qi)
        g, nrm = oracle.chunk_plaintexts(pb.pts, pb.slot, pb.N, k)
        f, r = oracle.server_chunk(pb.P, cts[qi], g, nrm, pb.key, int(pb.qids[qi]), k)
        out[m] = (oracle.rerandomize(pb.P, f, pks[qi], pb.key, int(pb.qids[qi]), k, b), r)
    return out


def _check_shares(stage, ctx, pb, sk, out, share, pairs):
    owner = np.array([q for q, _ in pairs])
    client = stage.decrypt_shares(ctx, sk, out, _dev(pb.qnorm2()[owner])).cpu().numpy()
    for m, (qi, k) in enumerate(pairs):
        ids = pb.slot[k * pb.N:(k + 1) * pb.N]
        real = ids >= 0
        tot = (client[m].astype(np.int64) + share[m].cpu().numpy()) % pb.P.t
        want = oracle.sqdist(pb.queries[qi], pb.pts[ids[real]])
        assert (tot[real] == want).all(), (m, qi, k)


CASES = [  # N, L, t_bits, n, d, Q, dtype
    (16, 2, 20, 40, 5, 2, "u8"),
    (1024, 1, 20, 3 * 1024 + 7, 6, 3, "u8"),
    (4096, 2, 25, 2 * 4096 + 77, 16, 2, "i8"),
    (8192, 3, 26, 8192 + 40, 12, 2, "u8"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-L{c[1]}-d{c[4]}-Q{c[5]}")
def test_private_form_matches_oracle(mods, case):
    nat, stage = mods
    N, L, tb, n, d, Q, dt = case
    pb = make_problem(N, L, tb, n, d, Q, dt, seed=500 + N)
    ctx, db, sk, ct, qids = _setup(nat, stage, pb)
    b = nat.sanns_flood_bits(ctx.handle)
    assert b == oracle.flood_bits(pb.P)
    pks, pkd = _public_keys(stage, ctx, pb, sk, 700)
    C = db.n_chunks
    D = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_FUSED, private=True)
    out, share = D.run(ct, pb.key, qids, pk=pkd)
    torch.cuda.synchronize()
    ctx.device_status()
    out_h, share_h = out.cpu().numpy().copy(), share.cpu().numpy().copy()
    M = Q * C
    rows = range(M) if M <= 8 else sorted(set([0, M - 1, C - 1, C] +
                                               list(np.random.default_rng(M).integers(0, M, 4))))
    want = _oracle_rows(pb, pks, [(m, divmod(m, C)) for m in rows], b, {})
    for m, (w_ct, w_r) in want.items():
        assert (out_h[m] == w_ct).all(), m
        assert (share_h[m] == w_r).all(), m
    # the graph form gives the same bytes; the plain form's shares are equal
    B = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED, private=True)
    for rep in range(2):
        bo, bs = B.run(ct, pb.key, qids, pk=pkd)
        torch.zeros(1 << 16, device="cuda").add_(1.0)
        torch.cuda.synchronize()
        assert (bo.cpu().numpy() == out_h).all() and (bs.cpu().numpy() == share_h).all(), rep
    po, ps = stage.distances(ctx, db, ct, pb.key, qids)
    assert (ps.cpu().numpy() == share_h).all()
    assert (po.cpu().numpy()[:, 1] != out_h[:, 1]).any()  # c1 re-randomised
    _check_shares(stage, ctx, pb, sk, out, share, [divmod(m, C) for m in range(M)])
    ctx.close()


def test_private_form_primes_away_from_2_54(mods):
    """50-bit primes take the general form of the flood residues' Horner
    step (a Shoup product by 2^32 mod q; primes 2^54 - delta with delta <
    2^22 take the short one): every output still equals the oracle's."""
    nat, stage = mods
    N = 1024
    qs = [oracle.rns_primes(N, i + 1, bits=50)[i] for i in range(2)]
    pb = make_problem(N, 2, 20, 2 * N + 13, 7, 2, "u8", seed=631, qs=qs)
    ctx, db, sk, ct, qids = _setup(nat, stage, pb)
    b = nat.sanns_flood_bits(ctx.handle)
    assert b == oracle.flood_bits(pb.P) and b > 32
    pks, pkd = _public_keys(stage, ctx, pb, sk, 900)
    C = db.n_chunks
    D = stage.Distances(ctx, db, pb.Q, mode=nat.SANNS_MODE_FUSED, private=True)
    out, share = D.run(ct, pb.key, qids, pk=pkd)
    torch.cuda.synchronize()
    ctx.device_status()
    M = pb.Q * C
    want = _oracle_rows(pb, pks, [(m, divmod(m, C)) for m in range(M)], b, {})
    for m, (w_ct, w_r) in want.items():
        assert (out[m].cpu().numpy() == w_ct).all(), m
        assert (share[m].cpu().numpy() == w_r).all(), m
    _check_shares(stage, ctx, pb, sk, out, share, [divmod(m, C) for m in range(M)])
    ctx.close()


def test_private_form_matrix_cores_and_work_lists(mods):
    """The matrix-core schedule and a work list give the oracle's outputs
    too, and a smaller flood width is honoured."""
    nat, stage = mods
    pb = make_problem(4096, 2, 25, 3 * 4096 + 11, 40, 4, "u8", seed=611)
    ctx, db, sk, ct, qids = _setup(nat, stage, pb, digits=True)
    pks, pkd = _public_keys(stage, ctx, pb, sk, 800)
    C = db.n_chunks
    b = nat.sanns_flood_bits(ctx.handle) - 7
    ctx.set_schedule(0, 0, nat.SANNS_SCHEDULE_MFMA)
    D = stage.Distances(ctx, db, pb.Q, mode=nat.SANNS_MODE_BATCHED, private=True)
    out, share = D.run(ct, pb.key, qids, pk=pkd, flood_bits=b)
    torch.cuda.synchronize()
    ctx.device_status()
    rows = [0, C + 1, 2 * C + 2, 4 * C - 1]
    want = _oracle_rows(pb, pks, [(m, divmod(m, C)) for m in rows], b, {})
    for m, (w_ct, w_r) in want.items():
        assert (out[m].cpu().numpy() == w_ct).all(), m
    ctx.set_schedule(0, 0, 22)
    vo, vs = D.__class__(ctx, db, pb.Q, mode=nat.SANNS_MODE_FUSED, private=True).run(
        ct, pb.key, qids, pk=pkd, flood_bits=b)
    assert torch.equal(vo.view(torch.int64), out.view(torch.int64))
    ctx.set_schedule(0, 0, 0)
    work = np.array([[3, 2], [0, 0], [1, 2], [3, 0]], dtype=np.uint32)
    W = stage.Distances(ctx, db, pb.Q, work=work, mode=nat.SANNS_MODE_BATCHED, private=True)
    wo, ws = W.run(ct, pb.key, qids, pk=pkd, flood_bits=b)
    torch.cuda.synchronize()
    want = _oracle_rows(pb, pks, [(m, (int(q), int(k))) for m, (q, k) in enumerate(work)], b, {})
    for m, (w_ct, w_r) in want.items():
        assert (wo[m].cpu().numpy() == w_ct).all(), m
        assert (ws[m].cpu().numpy() == w_r).all(), m
    _check_shares(stage, ctx, pb, sk, wo, ws, [tuple(int(x) for x in r) for r in work])
    ctx.close()


def test_private_form_limits(mods):
    nat, stage = mods
    pb = make_problem(4096, 2, 25, 100, 4, 1, "u8", seed=612)
    ctx, db, sk, ct, qids = _setup(nat, stage, pb)
    pkd = stage.public_key(ctx, sk, 5)[None].contiguous()
    D = stage.Distances(ctx, db, 1, mode=nat.SANNS_MODE_FUSED, private=True)
    with pytest.raises(nat.SannsError) as ei:
        D.run(ct, pb.key, qids, pk=pkd, flood_bits=nat.sanns_flood_bits(ctx.handle) + 1)
    assert ei.value.status == nat.SANNS_E_RANGE
    for mode in (nat.SANNS_MODE_PLAIN, nat.SANNS_MODE_PERSISTENT):
        P = stage.Distances(ctx, db, 1, mode=mode, private=True)
        with pytest.raises(nat.SannsError) as ei:
            P.run(ct, pb.key, qids, pk=pkd)
        assert ei.value.status == nat.SANNS_E_INVALID
    # a public-key residue out of range is caught on the device
    host = pkd.cpu().numpy().copy()
    host[0, 0, 0, 5] = np.uint64(pb.P.qs[0] + 5)
    D.run(ct, pb.key, qids, pk=_dev(host))
    with pytest.raises(nat.SannsError) as ei:
        ctx.device_status()
    assert ei.value.status == nat.SANNS_E_RANGE
    ctx.close()
