"""Degenerate inputs of the distance stage through every schedule (the
64-bit vector kernels, the int8 matrix cores, the fused single-query
kernel): the largest distance the plain modulus admits (every coordinate at
opposite ends of its range), a query equal to a database point (distance 0),
a database of one point (one chunk of N - 1 padding slots), one coordinate,
and an empty work list.  Sampled rows are compared with the oracle
coefficient for coefficient; every slot of every row is decrypted and
checked against the cleartext distance."""
import numpy as np
import pytest

import oracle
from problem import make_problem, oracle_query_ct, true_distances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MFMA, VECTOR = 81, 22


@pytest.fixture(scope="module")
def stage():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import stage as st
    return st


def _dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _setup(stage, pb):
    from paper_1904_02033_amd import native as nat
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    p.flags = (0 if pb.P.security_ok() else nat.SANNS_FLAG_INSECURE_TEST) | \
        nat.SANNS_FLAG_DIGIT_DB
    ctx = stage.Context(params=p)
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    return ctx, db, sk, ct, _dev(pb.qids)


def _check(stage, pb, ctx, sk, out, share, rows):
    """Oracle ciphertext coefficients and shares of the sampled rows; every
    slot of every row decrypts to its distance (padding: ||q||^2)."""
    N, C = pb.N, pb.C
    js = sorted(set([0, 1, N // 2, N - 1]))
    for m in rows:
        qi, k = divmod(m, C)
        g, nrm = oracle.chunk_plaintexts(pb.pts, pb.slot, N, k)
        sc, sr = oracle.server_coeffs(pb.P, oracle_query_ct(pb, qi), g, nrm, pb.key,
                                      int(pb.qids[qi]), k, js)
        assert (out[m][:, :, js] == sc).all(), m
        assert (share[m][js] == sr).all(), m
    owner = np.repeat(np.arange(pb.Q), C)
    qn2 = pb.qnorm2()
    client = stage.decrypt_shares(ctx, sk, _dev(out), _dev(qn2[owner])).cpu().numpy()
    for m in range(pb.Q * C):
        qi, k = divmod(m, C)
        dist = true_distances(pb, qi, k)
        tot = (client[m].astype(np.int64) + share[m].astype(np.int64)) % pb.P.t
        real = dist >= 0
        assert (tot[real] == dist[real]).all(), (m, qi, k)
        assert (tot[~real] == int(qn2[qi])).all(), (m, "padding")


def _all_schedules(stage, pb):
    """Outputs of the matrix-core, vector and fused schedules (equal bytes)."""
    from paper_1904_02033_amd import native as nat
    ctx, db, sk, ct, qids = _setup(stage, pb)
    res = []
    for variant, mode in ((MFMA, nat.SANNS_MODE_BATCHED), (VECTOR, nat.SANNS_MODE_BATCHED),
                          (0, nat.SANNS_MODE_FUSED)):
        ctx.set_schedule(0, 0, variant)
        D = stage.Distances(ctx, db, pb.Q, None, mode)
        out, share = D.run(ct, pb.key, qids)
        torch.cuda.synchronize()
        ctx.device_status()
        res.append((out.cpu().numpy().copy(), share.cpu().numpy().copy()))
    for o, s in res[1:]:
        assert (o == res[0][0]).all() and (s == res[0][1]).all()
    return ctx, sk, res[0]


@pytest.mark.parametrize("dt", ["u8", "i8"])
def test_largest_distance_and_zero_distance(stage, dt):
    """d = 128 with every coordinate at the opposite end of its range
    (d 255^2 = 8,323,200, just under the 25-bit t), and queries equal to
    database points; the rest of the database random."""
    N, d, n, Q = 4096, 128, 4096 + 300, 4
    lo, hi = (0, 255) if dt == "u8" else (-128, 127)
    npd = np.uint8 if dt == "u8" else np.int8
    g = np.random.default_rng(13)
    pts = g.integers(lo, hi + 1, (n, d)).astype(npd)
    pts[0] = lo
    pts[1] = hi
    qs = np.empty((Q, d), dtype=npd)
    qs[0] = hi                      # farthest from point 0
    qs[1] = lo                      # farthest from point 1
    qs[2] = pts[7]                  # equal to point 7
    qs[3] = pts[n - 1]              # equal to the last point
    pb = make_problem(N, 2, 25, 0, 0, 0, seed=17, points=pts, queries=qs)
    assert d * 255 * 255 < pb.P.t
    ctx, sk, (out, share) = _all_schedules(stage, pb)
    rows = sorted(set([0, pb.C - 1, pb.C, 2 * pb.C, 3 * pb.C + 1, pb.Q * pb.C - 1]))
    _check(stage, pb, ctx, sk, out, share, rows)
    # the extremes land where the slot map put the points
    owner = np.repeat(np.arange(pb.Q), pb.C)
    client = stage.decrypt_shares(ctx, sk, _dev(out), _dev(pb.qnorm2()[owner])).cpu().numpy()
    tot = (client.astype(np.int64) + share.astype(np.int64)) % pb.P.t
    where = {int(p): s for s, p in enumerate(pb.slot) if p >= 0}
    for qi, p, want in ((0, 0, d * 255 * 255), (1, 1, d * 255 * 255), (2, 7, 0), (3, n - 1, 0)):
        s = where[p]
        assert tot[qi * pb.C + s // N][s % N] == want, (qi, p)


def test_one_point_and_one_coordinate(stage):
    """A database of one point (one chunk, N - 1 padding slots) and d = 1,
    with two queries so that the matrix-core schedule runs."""
    pb = make_problem(4096, 2, 25, 1, 1, 2, "u8", seed=23)
    ctx, sk, (out, share) = _all_schedules(stage, pb)
    assert pb.C == 1
    _check(stage, pb, ctx, sk, out, share, range(pb.Q))


def test_empty_work_list_is_a_no_op(stage):
    """M = 0 returns at once and leaves the output buffers untouched."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(1024, 1, 20, 100, 3, 2, "u8", seed=29)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    out = torch.full((1, 2, 1, 1024), 7, dtype=torch.uint64, device="cuda")
    share = torch.full((1, 1024), 7, dtype=torch.uint32, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    nat.sanns_distances(ctx.handle, db.desc, ct.data_ptr(), pb.Q, pb.key, qids.data_ptr(),
                        np.zeros((1, 2), dtype=np.uint32)[:0], 0, nat.SANNS_MODE_FUSED,
                        out.data_ptr(), share.data_ptr(), ws.data_ptr(), ws.numel(), 0)
    torch.cuda.synchronize()
    ctx.device_status()
    assert (out == 7).all() and (share == 7).all()
