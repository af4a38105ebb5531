"""The seeded client helpers through the C ABI (sanns_keygen,
sanns_encrypt_query_seeded) against the oracle's independent samplers of the
same ChaCha20 definitions: key bit for bit, ciphertexts bit for bit, and the
seeded ciphertexts decrypting to the query and feeding the distance stage."""
import numpy as np
import pytest

import oracle
import synthdata

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1904_02033_amd import native as nat, stage
    return nat, stage


def _ctx(nat, stage, N, L, tb):
    P = oracle.Params(N, oracle.rns_primes(N, L), oracle.plain_modulus(N, tb))
    p = nat.sanns_params()
    p.N, p.L, p.t = N, L, P.t
    for l, q in enumerate(P.qs):
        p.q[l] = q
    if not P.security_ok():
        p.flags |= nat.SANNS_FLAG_INSECURE_TEST
    return P, stage.Context(params=p)


@pytest.mark.parametrize("N,L,tb,Q,d", [(16, 1, 8, 2, 3), (1024, 1, 20, 1, 5),
                                        (4096, 2, 25, 3, 7), (8192, 3, 26, 2, 4)])
def test_seeded_keygen_and_encryption_match_oracle(mods, N, L, tb, Q, d):
    nat, stage = mods
    P, ctx = _ctx(nat, stage, N, L, tb)
    sk = stage.keygen(ctx, 1234 + N)
    s_o = oracle.sample_secret(1234 + N, N)
    assert (sk.cpu().numpy() == s_o).all()
    g = np.random.default_rng(N)
    msgs = g.integers(-300, 300, (Q, d)).astype(np.int32)
    ct = stage.encrypt_query_seeded(ctx, sk, torch.as_tensor(msgs).cuda(), 99 + N)
    torch.cuda.synchronize()
    a_o, e_o = oracle.sample_encryption(P, 99 + N, Q, d)
    got = ct.cpu().numpy()
    for qi in range(Q):
        want = oracle.encrypt_constants(P, s_o, a_o[qi], e_o[qi], [int(x) for x in msgs[qi]])
        assert (got[qi] == want).all(), qi
    # the ciphertexts decrypt to the messages (oracle decryption)
    for qi, i in ((0, 0), (Q - 1, d - 1)):
        dec = oracle.decrypt(P, got[qi, i], s_o, coeffs=[0, 1, N - 1])
        assert dec == [int(msgs[qi, i]) % P.t, 0, 0]
    ctx.close()


def test_seeded_client_through_the_distance_stage(mods):
    """Seeded key and query encryption feed sanns_distances; the shares
    reconstruct the true distances at every slot."""
    nat, stage = mods
    N, L, tb, n, d, Q = 4096, 2, 25, 2 * 4096 + 100, 32, 3
    P, ctx = _ctx(nat, stage, N, L, tb)
    g = np.random.default_rng(5)
    pts = g.integers(0, 256, (n, d)).astype(np.uint8)
    qs = g.integers(0, 256, (Q, d)).astype(np.uint8)
    slot = synthdata.gen_slot_map(n, N, 6)
    db = stage.encode_db(ctx, pts, slot)
    sk = stage.keygen(ctx, 77)
    ct = stage.encrypt_query_seeded(ctx, sk, torch.as_tensor(qs.astype(np.int32)).cuda(), 78)
    key = synthdata.gen_mask_key(79)
    out, share = stage.distances(ctx, db, ct, key,
                                 torch.as_tensor(np.arange(Q, dtype=np.uint64)).cuda())
    C = db.n_chunks
    qn2 = ((qs.astype(np.int64) ** 2).sum(axis=1) % P.t).astype(np.uint32)
    client = stage.decrypt_shares(ctx, sk, out, torch.as_tensor(np.repeat(qn2, C)).cuda())
    torch.cuda.synchronize()
    ctx.device_status()
    tot = (client.cpu().numpy().astype(np.int64) + share.cpu().numpy()) % P.t
    for m in range(Q * C):
        qi, k = divmod(m, C)
        ids = slot[k * N:(k + 1) * N]
        real = ids >= 0
        assert (tot[m][real] == oracle.sqdist(qs[qi], pts[ids[real]])).all(), m
    ctx.close()
