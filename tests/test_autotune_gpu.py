"""Autotuner: every candidate schedule gives the same bytes, the fastest is
applied and cached, and a cache hit times nothing."""
import json

import numpy as np
import pytest

import oracle
from problem import make_problem, true_distances

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import autotune, native as nat, stage
    pb = make_problem(4096, 2, 25, 3 * 4096 + 17, 6, 3, "u8", seed=41)
    p = nat.sanns_params()
    p.N, p.L, p.t = pb.P.N, pb.P.L, pb.P.t
    for l, q in enumerate(pb.P.qs):
        p.q[l] = q
    ctx = stage.Context(params=p)
    db = stage.encode_db(ctx, pb.pts, pb.slot)
    sk = torch.as_tensor(pb.sk).cuda()
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(pb.queries.astype(np.int32)).cuda(),
                             torch.as_tensor(pb.a).cuda(), torch.as_tensor(pb.e).cuda())
    qids = torch.as_tensor(pb.qids).cuda()
    return dict(autotune=autotune, nat=nat, stage=stage, pb=pb, ctx=ctx, db=db, sk=sk, ct=ct,
                qids=qids)


def test_tune_all_pairs_picks_and_caches(world, tmp_path):
    at, nat, stage, pb = world["autotune"], world["nat"], world["stage"], world["pb"]
    ctx, db, ct, qids = world["ctx"], world["db"], world["ct"], world["qids"]
    cache = str(tmp_path / "tune.json")
    best, timed = at.tune(ctx, db, ct, pb.key, qids, reps=1, cache_path=cache)
    labels = [c.label() for c in timed]
    assert "persistent/51" in labels and "batched/lds22" in labels
    assert all(np.isfinite(c.ms) and c.ms > 0 for c in timed)
    assert best.ms == min(c.ms for c in timed)
    stored = json.load(open(cache))
    assert list(stored.values())[0]["variant"] == best.variant
    # the applied schedule still reconstructs the true distances
    D = stage.Distances(ctx, db, pb.Q, mode=best.mode)
    out, share = D.run(ct, pb.key, qids)
    qn = torch.as_tensor(np.repeat(pb.qnorm2(), pb.C)).cuda()
    client = stage.decrypt_shares(ctx, world["sk"], out, qn).cpu().numpy()
    share = share.cpu().numpy()
    for m in range(pb.Q * pb.C):
        qi, k = divmod(m, pb.C)
        dist = true_distances(pb, qi, k)
        real = dist >= 0
        tot = (client[m].astype(np.int64) + share[m]) % pb.P.t
        assert (tot[real] == dist[real]).all()
    # a cache hit returns the stored schedule without timing
    again, timed2 = at.tune(ctx, db, ct, pb.key, qids, reps=1, cache_path=cache)
    assert len(timed2) == 1 and again.variant == best.variant and again.mode == best.mode


def test_tune_work_list_uses_register_tiles(world):
    at, pb = world["autotune"], world["pb"]
    ctx, db, ct, qids = world["ctx"], world["db"], world["ct"], world["qids"]
    work = np.array([(0, 2), (1, 0), (1, 1), (2, 2), (0, 0)], dtype=np.uint32)
    best, timed = at.tune(ctx, db, ct, pb.key, qids, work=work, reps=1)
    labels = {c.label() for c in timed}
    assert "batched/tile2x4" in labels and "persistent/52" in labels
    assert best in timed
