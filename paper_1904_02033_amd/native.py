"""ctypes binding of libsanns.so (include/sanns.h), argument marshalling only.

Every function here has the name and argument order of its C entry point;
device pointers are passed as integers (e.g. ``tensor.data_ptr()``) and
streams as integer handles (``torch.cuda.current_stream().cuda_stream``).
A non-zero status raises SannsError with the library's message.  There is no
fallback: if the HIP library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsanns.so")

SANNS_OK = 0
SANNS_E_INVALID = -1
SANNS_E_PARAMS = -2
SANNS_E_RANGE = -3
SANNS_E_WORKSPACE = -4
SANNS_E_DEVICE = -5
SANNS_E_NOMEM = -6
STATUS_NAMES = {0: "SANNS_OK", -1: "SANNS_E_INVALID", -2: "SANNS_E_PARAMS",
                -3: "SANNS_E_RANGE", -4: "SANNS_E_WORKSPACE", -5: "SANNS_E_DEVICE",
                -6: "SANNS_E_NOMEM"}

SANNS_MAX_LIMBS = 4
SANNS_MAX_D = 4096
SANNS_FLAG_INSECURE_TEST = 1
SANNS_FLAG_DIGIT_DB = 2
SANNS_SCHEDULE_MFMA = 81
SANNS_U8, SANNS_I8, SANNS_SHARE32 = 0, 1, 2
SANNS_MODE_PLAIN, SANNS_MODE_FUSED, SANNS_MODE_BATCHED, SANNS_MODE_PERSISTENT = 0, 1, 2, 3

# Every exported symbol of include/sanns.h.
EXPORTS = [
    "sanns_params_derive", "sanns_ctx_create", "sanns_ctx_destroy",
    "sanns_last_error", "sanns_ctx_params", "sanns_db_bytes", "sanns_encode_db",
    "sanns_encrypt_query", "sanns_decrypt_shares", "sanns_distances_workspace",
    "sanns_distances", "sanns_device_status", "sanns_set_schedule",
    "sanns_profile_enable", "sanns_profile_read", "sanns_distances_noalloc",
    "sanns_keygen", "sanns_encrypt_query_seeded", "sanns_public_key", "sanns_distances_cp",
    "sanns_distances_cp_workspace", "sanns_flood_bits", "sanns_distances_gathered",
    "sanns_distances_gathered_workspace", "sanns_kmeans_workspace", "sanns_kmeans_init",
    "sanns_kmeans_assign", "sanns_kmeans_update", "sanns_slot_ranges",
]
SANNS_NOALLOC_SCRATCH_BYTES = 64 << 20
SANNS_N_PHASES = 7
PHASES = ["query_ntt", "masks", "mac", "intt_mask", "query_digits", "sums_transpose",
          "rerandomize"]


class SannsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sanns_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("q", ctypes.c_uint64 * SANNS_MAX_LIMBS), ("t", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class sanns_db(ctypes.Structure):
    _fields_ = [("mem", ctypes.c_void_p), ("bytes", ctypes.c_size_t),
                ("n_chunks", ctypes.c_uint32), ("d", ctypes.c_uint32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libsanns.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_1904_02033_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    st = ctypes.c_int
    L.sanns_params_derive.argtypes = [u32, u32, u32, ctypes.POINTER(sanns_params)]
    L.sanns_params_derive.restype = st
    L.sanns_ctx_create.argtypes = [ctypes.POINTER(sanns_params), i32, ctypes.POINTER(vp)]
    L.sanns_ctx_create.restype = st
    L.sanns_ctx_destroy.argtypes = [vp]
    L.sanns_ctx_destroy.restype = None
    L.sanns_last_error.argtypes = []
    L.sanns_last_error.restype = ctypes.c_char_p
    L.sanns_ctx_params.argtypes = [vp, ctypes.POINTER(sanns_params)]
    L.sanns_ctx_params.restype = st
    L.sanns_db_bytes.argtypes = [vp, u32, u32]
    L.sanns_db_bytes.restype = ctypes.c_size_t
    L.sanns_encode_db.argtypes = [vp, vp, i32, u64, vp, ctypes.POINTER(sanns_db), vp]
    L.sanns_encode_db.restype = st
    L.sanns_encrypt_query.argtypes = [vp, vp, vp, u32, u32, vp, vp, vp, vp]
    L.sanns_encrypt_query.restype = st
    L.sanns_keygen.argtypes = [vp, u64, vp, vp]
    L.sanns_keygen.restype = st
    L.sanns_encrypt_query_seeded.argtypes = [vp, vp, vp, u32, u32, u64, vp, vp]
    L.sanns_encrypt_query_seeded.restype = st
    L.sanns_public_key.argtypes = [vp, vp, u64, vp, vp]
    L.sanns_public_key.restype = st
    L.sanns_distances_cp.argtypes = [vp, ctypes.POINTER(sanns_db), vp, u32, ctypes.c_char_p,
                                     vp, vp, u32, vp, u32, i32, vp, vp, vp, ctypes.c_size_t,
                                     vp]
    L.sanns_distances_cp.restype = st
    L.sanns_distances_cp_workspace.argtypes = [vp, ctypes.POINTER(sanns_db), u32, u32, i32]
    L.sanns_distances_cp_workspace.restype = ctypes.c_size_t
    L.sanns_distances_gathered.argtypes = [vp, vp, i32, u64, u32, vp, vp, vp, u32,
                                           ctypes.POINTER(sanns_db), vp, u32, ctypes.c_char_p,
                                           vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sanns_distances_gathered.restype = st
    L.sanns_distances_gathered_workspace.argtypes = [vp, u32, u32, u32,
                                                     ctypes.POINTER(sanns_db)]
    L.sanns_distances_gathered_workspace.restype = ctypes.c_size_t
    L.sanns_slot_ranges.argtypes = [vp, vp, vp, u32, vp, u64, vp]
    L.sanns_slot_ranges.restype = st
    L.sanns_kmeans_workspace.argtypes = [u32, u32]
    L.sanns_kmeans_workspace.restype = ctypes.c_size_t
    L.sanns_kmeans_init.argtypes = [vp, u64, u32, vp, u32, vp, vp, vp]
    L.sanns_kmeans_init.restype = st
    L.sanns_kmeans_assign.argtypes = [vp, u64, u32, vp, u32, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.sanns_kmeans_assign.restype = st
    L.sanns_kmeans_update.argtypes = [vp, u64, u32, vp, u32, vp, vp, vp, ctypes.c_size_t, vp]
    L.sanns_kmeans_update.restype = st
    L.sanns_flood_bits.argtypes = [vp]
    L.sanns_flood_bits.restype = u32
    L.sanns_decrypt_shares.argtypes = [vp, vp, vp, u32, vp, vp, vp]
    L.sanns_decrypt_shares.restype = st
    L.sanns_distances_workspace.argtypes = [vp, ctypes.POINTER(sanns_db), u32, u32, i32]
    L.sanns_distances_workspace.restype = ctypes.c_size_t
    L.sanns_distances.argtypes = [vp, ctypes.POINTER(sanns_db), vp, u32, ctypes.c_char_p,
                                  vp, vp, u32, i32, vp, vp, vp, ctypes.c_size_t, vp]
    L.sanns_distances.restype = st
    L.sanns_distances_noalloc.argtypes = [vp, ctypes.POINTER(sanns_db), vp, u32,
                                          ctypes.c_char_p, vp, vp, vp, vp]
    L.sanns_distances_noalloc.restype = st
    L.sanns_device_status.argtypes = [vp, vp]
    L.sanns_device_status.restype = st
    L.sanns_set_schedule.argtypes = [vp, i32, i32, i32]
    L.sanns_set_schedule.restype = st
    L.sanns_profile_enable.argtypes = [vp, i32]
    L.sanns_profile_enable.restype = st
    L.sanns_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int)]
    L.sanns_profile_read.restype = st
    _lib = L
    return L


def _check(status: int):
    if status != SANNS_OK:
        raise SannsError(status, load().sanns_last_error().decode())


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------

def sanns_params_derive(N: int, L: int, t_bits: int) -> sanns_params:
    p = sanns_params()
    _check(load().sanns_params_derive(N, L, t_bits, ctypes.byref(p)))
    return p


def sanns_ctx_create(p: sanns_params, device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load().sanns_ctx_create(ctypes.byref(p), device, ctypes.byref(h)))
    return h.value


def sanns_ctx_destroy(ctx: int) -> None:
    load().sanns_ctx_destroy(ctx)


def sanns_ctx_params(ctx: int) -> sanns_params:
    p = sanns_params()
    _check(load().sanns_ctx_params(ctx, ctypes.byref(p)))
    return p


def sanns_db_bytes(ctx: int, n_chunks: int, d: int) -> int:
    return load().sanns_db_bytes(ctx, n_chunks, d)


def sanns_encode_db(ctx: int, points: int, dtype: int, n: int, slot_point: int,
                    db: sanns_db, stream: int = 0) -> None:
    _check(load().sanns_encode_db(ctx, points, dtype, n, slot_point, ctypes.byref(db),
                                  stream))


def sanns_encrypt_query(ctx: int, sk: int, msgs: int, Q: int, d: int, a: int, e: int,
                        ct_out: int, stream: int = 0) -> None:
    _check(load().sanns_encrypt_query(ctx, sk, msgs, Q, d, a, e, ct_out, stream))


def sanns_keygen(ctx: int, seed: int, sk: int, stream: int = 0) -> None:
    _check(load().sanns_keygen(ctx, seed, sk, stream))


def sanns_encrypt_query_seeded(ctx: int, sk: int, msgs: int, Q: int, d: int, enc_seed: int,
                               ct_out: int, stream: int = 0) -> None:
    _check(load().sanns_encrypt_query_seeded(ctx, sk, msgs, Q, d, enc_seed, ct_out, stream))


def sanns_public_key(ctx: int, sk: int, seed: int, pk: int, stream: int = 0) -> None:
    _check(load().sanns_public_key(ctx, sk, seed, pk, stream))


def sanns_distances_cp(ctx: int, db: sanns_db, ct_in: int, Q: int, mask_key: bytes,
                       query_ids: int, pk: int, flood_bits: int, work, M: int, mode: int,
                       ct_out: int, server_share: int, workspace: int, ws_bytes: int,
                       stream: int = 0) -> None:
    if len(mask_key) != 32:
        raise ValueError("mask_key must be 32 bytes")
    wp = None if work is None else work.ctypes.data_as(ctypes.c_void_p)
    _check(load().sanns_distances_cp(ctx, ctypes.byref(db), ct_in, Q, mask_key, query_ids, pk,
                                     flood_bits, wp, M, mode, ct_out, server_share, workspace,
                                     ws_bytes, stream))


def sanns_distances_cp_workspace(ctx: int, db: sanns_db, Q: int, M: int, mode: int) -> int:
    return load().sanns_distances_cp_workspace(ctx, ctypes.byref(db), Q, M, mode)


def sanns_distances_gathered(ctx: int, points: int, dtype: int, n: int, d: int,
                             norm_shares: int, slot_point: int, row_query, M: int, tail,
                             ct_in: int, Q: int, mask_key: bytes, query_ids: int, ct_out: int,
                             server_share: int, workspace: int, ws_bytes: int,
                             stream: int = 0) -> None:
    """``row_query`` is a C-contiguous host numpy uint32 array [M]; ``tail``
    a sanns_db or None."""
    if len(mask_key) != 32:
        raise ValueError("mask_key must be 32 bytes")
    _check(load().sanns_distances_gathered(
        ctx, points, dtype, n, d, norm_shares, slot_point,
        row_query.ctypes.data_as(ctypes.c_void_p), M,
        None if tail is None else ctypes.byref(tail), ct_in, Q, mask_key, query_ids, ct_out,
        server_share, workspace, ws_bytes, stream))


def sanns_distances_gathered_workspace(ctx: int, d: int, Q: int, M: int, tail=None) -> int:
    return load().sanns_distances_gathered_workspace(
        ctx, d, Q, M, None if tail is None else ctypes.byref(tail))


def sanns_slot_ranges(start: int, length: int, off: int, R: int, slot_point: int, total: int,
                      stream: int = 0) -> None:
    _check(load().sanns_slot_ranges(start, length, off, R, slot_point, total, stream))


def sanns_kmeans_workspace(k: int, d: int) -> int:
    return load().sanns_kmeans_workspace(k, d)


def sanns_kmeans_init(points: int, n: int, d: int, idx: int, k: int, centers: int, bad: int,
                      stream: int = 0) -> None:
    _check(load().sanns_kmeans_init(points, n, d, idx, k, centers, bad, stream))


def sanns_kmeans_assign(points: int, n: int, d: int, centers: int, k: int, prev: int,
                        assign: int, changed: int, workspace: int, ws_bytes: int,
                        stream: int = 0) -> None:
    _check(load().sanns_kmeans_assign(points, n, d, centers, k, prev, assign, changed,
                                      workspace, ws_bytes, stream))


def sanns_kmeans_update(points: int, n: int, d: int, assign: int, k: int, centers: int,
                        counts: int, workspace: int, ws_bytes: int, stream: int = 0) -> None:
    _check(load().sanns_kmeans_update(points, n, d, assign, k, centers, counts, workspace,
                                      ws_bytes, stream))


def sanns_flood_bits(ctx: int) -> int:
    return load().sanns_flood_bits(ctx)


def sanns_decrypt_shares(ctx: int, sk: int, ct: int, M: int, qnorm2: int,
                         client_share: int, stream: int = 0) -> None:
    _check(load().sanns_decrypt_shares(ctx, sk, ct, M, qnorm2, client_share, stream))


def sanns_distances_noalloc(ctx: int, db: sanns_db, ct_in: int, Q: int, mask_key: bytes,
                            query_ids: int, ct_out: int, server_share: int,
                            stream: int = 0) -> None:
    if len(mask_key) != 32:
        raise ValueError("mask_key must be 32 bytes")
    _check(load().sanns_distances_noalloc(ctx, ctypes.byref(db), ct_in, Q, mask_key,
                                          query_ids, ct_out, server_share, stream))


def sanns_distances_workspace(ctx: int, db: sanns_db, Q: int, M: int, mode: int) -> int:
    return load().sanns_distances_workspace(ctx, ctypes.byref(db), Q, M, mode)


def sanns_distances(ctx: int, db: sanns_db, ct_in: int, Q: int, mask_key: bytes,
                    query_ids: int, work, M: int, mode: int, ct_out: int,
                    server_share: int, workspace: int, ws_bytes: int,
                    stream: int = 0) -> None:
    """``work`` is None or a C-contiguous host numpy uint32 array [M][2]."""
    if len(mask_key) != 32:
        raise ValueError("mask_key must be 32 bytes")
    wp = None if work is None else work.ctypes.data_as(ctypes.c_void_p)
    _check(load().sanns_distances(ctx, ctypes.byref(db), ct_in, Q, mask_key, query_ids, wp,
                                  M, mode, ct_out, server_share, workspace, ws_bytes,
                                  stream))


def sanns_device_status(ctx: int, stream: int = 0) -> None:
    _check(load().sanns_device_status(ctx, stream))


def sanns_set_schedule(ctx: int, lds_variant: int, qt: int, ct: int) -> None:
    _check(load().sanns_set_schedule(ctx, lds_variant, qt, ct))


def sanns_profile_enable(ctx: int, on: bool) -> None:
    _check(load().sanns_profile_enable(ctx, 1 if on else 0))


def sanns_profile_read(ctx: int):
    """Returns ({phase: mean ms}, calls)."""
    ms = (ctypes.c_double * SANNS_N_PHASES)()
    calls = ctypes.c_int(0)
    _check(load().sanns_profile_read(ctx, ms, ctypes.byref(calls)))
    return dict(zip(PHASES, list(ms))), calls.value
