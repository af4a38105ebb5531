"""The matrix-core schedule of the all-pairs multiply-accumulate
(SANNS_SCHEDULE_MFMA: int8 MFMA on the signed base-256 digits of both
operands) against the oracle, with query, chunk and coordinate counts that
leave ragged row tiles, chunk tiles and 64-coordinate steps; against the
64-bit vector schedule bit for bit; graph replays; and the host-side limits."""
import numpy as np
import pytest

import oracle
from problem import make_problem, oracle_query_ct, true_distances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MFMA = 81


@pytest.fixture(scope="module")
def stage():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import stage as st
    return st


def _ctx(stage, pb, digits=True):
    from paper_1904_02033_amd import native as nat
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    p.flags = 0 if pb.P.security_ok() else nat.SANNS_FLAG_INSECURE_TEST
    if digits:
        p.flags |= nat.SANNS_FLAG_DIGIT_DB
    return stage.Context(params=p)


def _dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def _setup(stage, pb, digits=True):
    ctx = _ctx(stage, pb, digits)
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    sk = _dev(pb.sk)
    ct = stage.encrypt_query(ctx, sk, _dev(pb.queries, torch.int32), _dev(pb.a), _dev(pb.e))
    return ctx, db, sk, ct, _dev(pb.qids)


def _run(stage, ctx, db, pb, ct, qids, mode, variant):
    ctx.set_schedule(0, 0, variant)
    D = stage.Distances(ctx, db, pb.Q, None, mode)
    out, share = D.run(ct, pb.key, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    return out.cpu().numpy().copy(), share.cpu().numpy().copy()


def _check_rows(stage, pb, ctx, sk, out, share, rows, n_coeffs=16):
    """Oracle server shares and sampled ciphertext coefficients of the given
    output rows, and client + server = ||q - p||^2 at every slot."""
    N, C = pb.N, pb.C
    js = sorted(set([0, 1, N - 1] + list(np.random.default_rng(N + 7).integers(0, N, n_coeffs))))
    cts = {}
    for m in rows:
        qi, k = divmod(m, C)
        if qi not in cts:
            cts[qi] = oracle_query_ct(pb, qi)
        g, nrm = oracle.chunk_plaintexts(pb.pts, pb.slot, N, k)
        sc, sr = oracle.server_coeffs(pb.P, cts[qi], g, nrm, pb.key, int(pb.qids[qi]), k, js)
        assert (out[m][:, :, js] == sc).all(), m
        assert (share[m][js] == sr).all(), m
    owner = np.repeat(np.arange(pb.Q), C)
    client = stage.decrypt_shares(ctx, sk, _dev(out), _dev(pb.qnorm2()[owner])).cpu().numpy()
    for m in range(pb.Q * C):
        qi, k = divmod(m, C)
        dist = true_distances(pb, qi, k)
        tot = (client[m].astype(np.int64) + share[m].astype(np.int64)) % pb.P.t
        real = dist >= 0
        assert (tot[real] == dist[real]).all(), (m, qi, k)


# (N, L, t_bits, n, d, Q, dtype): ragged against the 64-row and 16-row tiles,
# the 32- and 16-chunk tiles and the 64-coordinate steps; the ring degrees
# 64 .. 512 cover every form of the split transforms (the forward head ends
# and the inverse tail starts at a narrow pass of 2, 3, 4 or 1 bits)
CASES = [
    (4096, 2, 25, 2 * 4096 + 77, 7, 5, "u8"),
    (8192, 3, 26, 8192 + 5, 100, 3, "i8"),
    (2048, 1, 20, 3 * 2048 + 1, 8, 9, "u8"),
    (16384, 3, 26, 16384 + 100, 128, 2, "i8"),
    (64, 2, 22, 64 * 9 + 5, 4, 5, "u8"),
    (128, 2, 22, 128 * 5 + 3, 5, 7, "i8"),
    (256, 1, 25, 256 * 40 + 1, 70, 3, "u8"),
    (512, 2, 25, 512 * 3, 33, 4, "i8"),
    # the 1M x 96 workload's ring and dimension (a 32-coordinate last step),
    # 80 rows in two row tiles
    (8192, 3, 26, 3 * 8192 + 17, 96, 40, "i8"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"N{c[0]}-d{c[4]}-Q{c[5]}-{c[6]}")
def test_mfma_matches_oracle_and_vector_schedule(stage, case):
    from paper_1904_02033_amd import native as nat
    N, L, tb, n, d, Q, dt = case
    pb = make_problem(N, L, tb, n, d, Q, dt, seed=N + d)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    out, share = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_FUSED, MFMA)
    M = pb.Q * pb.C
    # oracle coefficients of every row, or of a sample when there are many
    # (every row is still compared with the vector schedule and decrypted)
    rows = range(M) if M <= 64 else sorted(
        set([0, M - 1] + list(np.random.default_rng(M).integers(0, M, 14))))
    _check_rows(stage, pb, ctx, sk, out, share, rows)
    vo, vs = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_FUSED, 22)
    assert (vo == out).all() and (vs == share).all()


@pytest.mark.parametrize("dt", ["u8", "i8"])
def test_power_of_two_t(stage, dt):
    """t = 2^24 (the paper's kind of plain modulus, Section 5): both
    schedules agree with the oracle and with each other, and the shares
    reconstruct every distance."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(4096, 2, 25, 2 * 4096 + 33, 100, 4, dt, seed=41, t=1 << 24)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    assert ctx.t == 1 << 24
    out, share = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_BATCHED, MFMA)
    _check_rows(stage, pb, ctx, sk, out, share, range(pb.Q * pb.C), n_coeffs=8)
    vo, vs = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_FUSED, 22)
    assert (vo == out).all() and (vs == share).all()


@pytest.mark.parametrize("bits", [(50, 50), (54, 50), (54, 52)])
def test_primes_away_from_2_54(stage, bits):
    """The fold of the digit sums has two forms: a short one that uses
    2^54 = delta (mod q) when every prime is 2^54 - delta with delta < 2^22
    (the primes the workloads use), and a general one with Shoup products.
    Primes of 50 and 52 bits, alone or beside a prime just below 2^54, take
    the general form; both agree with the oracle and the vector schedule."""
    from paper_1904_02033_amd import native as nat
    N = 4096
    qs = [oracle.rns_primes(N, i + 1, bits=b)[i] for i, b in enumerate(bits)]
    assert any((1 << 54) - q >= 1 << 22 for q in qs)
    pb = make_problem(N, 2, 25, 2 * N + 51, 100, 5, "i8", seed=43, qs=qs)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    out, share = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_BATCHED, MFMA)
    _check_rows(stage, pb, ctx, sk, out, share, range(pb.Q * pb.C), n_coeffs=8)
    vo, vs = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_FUSED, 22)
    assert (vo == out).all() and (vs == share).all()


def test_mfma_many_tiles_equals_vector_schedule(stage):
    """66 rows (two row tiles, the second with 2 rows) x 33 chunks (two chunk
    tiles, the second with one chunk), d = 128: every output equal to the
    vector schedule's, oracle rows sampled, shares decrypt to distances."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(4096, 2, 25, 33 * 4096 - 50, 128, 33, "u8", seed=91)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    out, share = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_BATCHED, MFMA)
    vo, vs = _run(stage, ctx, db, pb, ct, qids, nat.SANNS_MODE_BATCHED, 22)
    assert (vo == out).all() and (vs == share).all()
    g = np.random.default_rng(5)
    rows = sorted(set([0, pb.Q * pb.C - 1, 32, 33 * 32] + list(g.integers(0, pb.Q * pb.C, 6))))
    _check_rows(stage, pb, ctx, sk, out, share, rows, n_coeffs=6)


def test_mfma_graph_replays_pick_up_new_inputs(stage):
    from paper_1904_02033_amd import native as nat
    pb = make_problem(4096, 2, 25, 3 * 4096 + 11, 20, 4, "u8", seed=31)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    ctx.set_schedule(0, 0, MFMA)
    B = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_BATCHED)
    want = None
    for rep in range(4):
        if rep in (0, 2):
            if rep == 2:
                ct.copy_(ct.flip(0).contiguous())
                qids.copy_(qids.flip(0).contiguous())
            ctx.set_schedule(0, 0, 22)
            F = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_FUSED)
            fo, fs = F.run(ct, pb.key, qids)
            torch.cuda.synchronize()
            want = (fo.cpu().numpy().copy(), fs.cpu().numpy().copy())
            ctx.set_schedule(0, 0, MFMA)
        o, s = B.run(ct, pb.key, qids)
        torch.zeros(1 << 20, device="cuda").add_(1.0)  # unrelated eager work
        torch.cuda.synchronize()
        ctx.device_status()
        assert (o.cpu().numpy() == want[0]).all() and (s.cpu().numpy() == want[1]).all(), rep


def test_mfma_default_and_limits(stage):
    from paper_1904_02033_amd import native as nat
    # without the flag the schedule cannot be selected
    pb = make_problem(4096, 2, 25, 100, 8, 2, "u8", seed=3)
    ctx = _ctx(stage, pb, digits=False)
    with pytest.raises(nat.SannsError) as ei:
        ctx.set_schedule(0, 0, MFMA)
    assert ei.value.status == nat.SANNS_E_INVALID
    # the flag adds the digit form to the database size
    ctxd = _ctx(stage, pb, digits=True)
    plain = nat.sanns_db_bytes(ctx.handle, 3, 100)
    assert nat.sanns_db_bytes(ctxd.handle, 3, 100) == plain + 2 * 4096 * 3 * (7 * 128 + 16) + 65536
    assert nat.sanns_db_bytes(ctxd.handle, 3, 200) == nat.sanns_db_bytes(ctx.handle, 3, 200)
    # d > 128: no digit form; forcing the schedule is a host error, the
    # default falls back to the vector schedule
    wide = make_problem(4096, 2, 26, 40, 150, 2, "u8", seed=4)
    ctx, db, sk, ct, qids = _setup(stage, wide)
    ctx.set_schedule(0, 0, MFMA)
    D = stage.Distances(ctx, db, 2, None, nat.SANNS_MODE_FUSED)
    with pytest.raises(nat.SannsError) as ei:
        D.run(ct, wide.key, qids)
    assert ei.value.status == nat.SANNS_E_INVALID
    ctx.set_schedule(0, 0, 0)
    out, share = D.run(ct, wide.key, qids)
    torch.cuda.synchronize()
    ctx.device_status()
    want = oracle.masks(wide.key, int(wide.qids[1]), 0, wide.P.t, wide.N)
    assert (share[1].cpu().numpy() == want).all()


def test_profile_phases_split_by_schedule(stage):
    """Per-phase timing: the matrix-core schedule reports its digit and sums
    transposes as phases of their own (the masks drawn inside the sums
    transpose); the vector schedule leaves them 0."""
    from paper_1904_02033_amd import native as nat
    pb = make_problem(8192, 3, 26, 3 * 8192, 64, 8, "u8", seed=7)
    ctx, db, sk, ct, qids = _setup(stage, pb)
    for variant, extra in ((MFMA, True), (22, False)):
        ctx.set_schedule(0, 0, variant)
        D = stage.Distances(ctx, db, pb.Q, None, nat.SANNS_MODE_BATCHED)
        D.run(ct, pb.key, qids)
        nat.sanns_profile_enable(ctx.handle, True)
        for _ in range(2):
            D.run(ct, pb.key, qids)
        ph, calls = nat.sanns_profile_read(ctx.handle)
        nat.sanns_profile_enable(ctx.handle, False)
        ctx.device_status()
        assert calls == 2 and set(ph) == set(nat.PHASES)
        for k in ("query_ntt", "mac", "intt_mask"):
            assert ph[k] > 0, (variant, k)
        for k in ("query_digits", "sums_transpose"):
            assert (ph[k] > 0) == extra or (not extra and ph[k] < 0.05), (variant, k, ph[k])
        # the masks phase: a kernel of its own only in the vector schedule;
        # in the matrix-core one it brackets no work, like the re-randomisation
        # phase of a call without public keys
        if extra:
            assert ph["masks"] < ph["rerandomize"] + 0.01, (variant, ph)
        else:
            assert ph["masks"] > 0, (variant, ph)
