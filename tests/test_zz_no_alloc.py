"""sanns_distances_noalloc (the entry point for callers that cannot allocate)
against sanns_distances on the same inputs, through the C ABI: two calls in
a row, the second with a smaller input; the matrix-core schedule through the
scratch array; the size limit; and no device memory taken by the call."""
import numpy as np
import pytest

import oracle
from problem import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import native as nat, stage
    return nat, stage


def _ctx(nat, stage, pb, digits=False):
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    if not pb.P.security_ok():
        p.flags |= nat.SANNS_FLAG_INSECURE_TEST
    if digits:
        p.flags |= nat.SANNS_FLAG_DIGIT_DB
    return stage.Context(params=p)


def _inputs(stage, ctx, pb):
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x)).cuda()
    ct = stage.encrypt_query(ctx, dev(pb.sk), dev(pb.queries.astype(np.int32)), dev(pb.a),
                             dev(pb.e))
    return db, ct, dev(pb.qids)


def _noalloc(nat, ctx, db, ct, pb, qids, stream):
    M = pb.Q * db.n_chunks
    out = torch.empty((M, 2, ctx.L, ctx.N), dtype=torch.uint64, device="cuda")
    share = torch.empty((M, ctx.N), dtype=torch.uint32, device="cuda")
    nat.sanns_distances_noalloc(ctx.handle, db.desc, ct.data_ptr(), pb.Q, pb.key,
                                qids.data_ptr(), out.data_ptr(), share.data_ptr(),
                                stream.cuda_stream)
    return out, share


def _check(nat, stage, ctx, db, ct, pb, qids):
    stream = torch.cuda.current_stream()
    got_o, got_s = _noalloc(nat, ctx, db, ct, pb, qids, stream)
    want_o, want_s = stage.distances(ctx, db, ct, pb.key, qids, mode=nat.SANNS_MODE_FUSED)
    torch.cuda.synchronize()
    ctx.device_status()
    assert torch.equal(got_o.view(torch.int64), want_o.view(torch.int64))
    assert torch.equal(got_s.view(torch.int32), want_s.view(torch.int32))
    # and the shares of the first and last rows are the oracle's masks
    C = db.n_chunks
    for m in (0, pb.Q * C - 1):
        qi, k = divmod(m, C)
        r = oracle.masks(pb.key, int(pb.qids[qi]), k, pb.P.t, pb.N)
        assert (got_s[m].cpu().numpy() == r).all(), m


def test_noalloc_equals_distances_two_calls_second_smaller(mods):
    nat, stage = mods
    big = make_problem(4096, 2, 25, 3 * 4096 + 77, 40, 3, "u8", seed=301)
    small = make_problem(4096, 2, 25, 4096 + 5, 16, 1, "u8", seed=302)
    ctx = _ctx(nat, stage, big)
    for pb in (big, small):
        db, ct, qids = _inputs(stage, ctx, pb)
        _check(nat, stage, ctx, db, ct, pb, qids)
    ctx.close()


def test_noalloc_matrix_core_schedule_and_full_ring(mods):
    """A digit database with the matrix-core schedule forced (its digit and
    sums regions come from the scratch array too: the sums of 64-row x
    64-chunk tiles fit it up to N = 2048), then one query at N = 8192, L = 3,
    d = 128: the 1M x 128 scan's ring and width."""
    nat, stage = mods
    pb = make_problem(512, 2, 23, 40 * 512 + 9, 40, 4, "i8", seed=303)
    ctx = _ctx(nat, stage, pb, digits=True)
    ctx.set_schedule(0, 0, nat.SANNS_SCHEDULE_MFMA)
    db, ct, qids = _inputs(stage, ctx, pb)
    _check(nat, stage, ctx, db, ct, pb, qids)
    ctx.close()
    pb = make_problem(8192, 3, 25, 8192 + 40, 128, 1, "u8", seed=304)
    ctx = _ctx(nat, stage, pb)
    db, ct, qids = _inputs(stage, ctx, pb)
    _check(nat, stage, ctx, db, ct, pb, qids)
    # repeated calls take no device memory
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    outs = _noalloc(nat, ctx, db, ct, pb, qids, stream)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        nat.sanns_distances_noalloc(ctx.handle, db.desc, ct.data_ptr(), pb.Q, pb.key,
                                    qids.data_ptr(), outs[0].data_ptr(), outs[1].data_ptr(),
                                    stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    ctx.close()


def test_noalloc_rejects_calls_beyond_the_scratch(mods):
    nat, stage = mods
    pb = make_problem(8192, 3, 25, 8192, 128, 2, "u8", seed=305)
    ctx = _ctx(nat, stage, pb)
    db, ct, qids = _inputs(stage, ctx, pb)
    need = nat.sanns_distances_workspace(ctx.handle, db.desc, 2, 2 * db.n_chunks,
                                         nat.SANNS_MODE_FUSED)
    assert need > nat.SANNS_NOALLOC_SCRATCH_BYTES
    out = torch.empty((2 * db.n_chunks, 2, 3, 8192), dtype=torch.uint64, device="cuda")
    share = torch.empty((2 * db.n_chunks, 8192), dtype=torch.uint32, device="cuda")
    with pytest.raises(nat.SannsError) as ei:
        nat.sanns_distances_noalloc(ctx.handle, db.desc, ct.data_ptr(), 2, pb.key,
                                    qids.data_ptr(), out.data_ptr(), share.data_ptr(), 0)
    assert ei.value.status == nat.SANNS_E_WORKSPACE
    assert "scratch" in str(ei.value)
    ctx.close()
