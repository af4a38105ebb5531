"""Torch-tensor front end of the C ABI (argument marshalling only).

PyTorch provides device memory and streams; every step of the distance stage
runs in the HIP kernels of libsanns.so behind ``native``.  Shapes follow
include/sanns.h.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import native as nat


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class Context:
    """A parameter set bound to one device (sanns_ctx)."""

    def __init__(self, N: int = 8192, L: int = 3, t_bits: int = 25, device: int = 0,
                 params: Optional[nat.sanns_params] = None, insecure: bool = False):
        p = params if params is not None else nat.sanns_params_derive(N, L, t_bits)
        if insecure:
            p.flags |= nat.SANNS_FLAG_INSECURE_TEST
        self.device = device
        self.handle = nat.sanns_ctx_create(p, device)
        self.params = nat.sanns_ctx_params(self.handle)
        self.N, self.L, self.t = self.params.N, self.params.L, self.params.t
        self.qs = [self.params.q[l] for l in range(self.L)]

    def close(self):
        if self.handle:
            torch.cuda.synchronize(self.device)
            nat.sanns_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_schedule(self, qt: int = 0, ct: int = 0, lds_variant: int = 0):
        nat.sanns_set_schedule(self.handle, lds_variant, qt, ct)

    def device_status(self, stream=None):
        nat.sanns_device_status(self.handle, _stream(stream))


@dataclasses.dataclass
class Database:
    mem: torch.Tensor          # uint8 device buffer owning the resident form
    desc: nat.sanns_db
    n: int
    d: int
    n_chunks: int
    slot_point: torch.Tensor   # int64 [n_chunks * N] on the device

    @property
    def nbytes(self) -> int:
        return self.desc.bytes


def linear_slot_map(n: int, N: int, perm: np.ndarray) -> np.ndarray:
    """Slot s of chunk k holds point perm[kN + s]; padding slots hold -1."""
    C = (n + N - 1) // N
    m = np.full(C * N, -1, dtype=np.int64)
    m[:n] = perm
    return m


def encode_db(ctx: Context, points, slot_point: np.ndarray, stream=None) -> Database:
    """sanns_encode_db on device copies of ``points`` ([n][d] uint8/int8)
    and the slot map."""
    dev = torch.device("cuda", ctx.device)
    pts = torch.as_tensor(points).to(dev).contiguous()
    if pts.dtype == torch.uint8:
        dtype = nat.SANNS_U8
    elif pts.dtype == torch.int8:
        dtype = nat.SANNS_I8
    else:
        raise ValueError("points must be uint8 or int8")
    n, d = pts.shape
    if len(slot_point) % ctx.N:
        raise ValueError("slot map length must be a multiple of N")
    C = len(slot_point) // ctx.N
    sp = torch.as_tensor(np.ascontiguousarray(slot_point, dtype=np.int64)).to(dev)
    nbytes = nat.sanns_db_bytes(ctx.handle, C, d)
    mem = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    desc = nat.sanns_db(mem.data_ptr(), nbytes, C, d)
    nat.sanns_encode_db(ctx.handle, pts.data_ptr(), dtype, n, sp.data_ptr(), desc,
                        _stream(stream))
    return Database(mem, desc, n, d, C, sp)


def encrypt_query(ctx: Context, sk: torch.Tensor, msgs: torch.Tensor, a: torch.Tensor,
                  e: torch.Tensor, stream=None) -> torch.Tensor:
    """Client-side encryption of Q queries: returns ct [Q][d][2][L][N] uint64."""
    Q, d = msgs.shape
    ct = torch.empty((Q, d, 2, ctx.L, ctx.N), dtype=torch.uint64, device=msgs.device)
    nat.sanns_encrypt_query(ctx.handle, _ptr(sk), _ptr(msgs), Q, d, _ptr(a), _ptr(e),
                            _ptr(ct), _stream(stream))
    return ct


def keygen(ctx: Context, seed: int, stream=None) -> torch.Tensor:
    """Client secret key [N] int8 drawn from a seed (sanns_keygen)."""
    sk = torch.empty(ctx.N, dtype=torch.int8, device=torch.device("cuda", ctx.device))
    nat.sanns_keygen(ctx.handle, seed, _ptr(sk), _stream(stream))
    return sk


def encrypt_query_seeded(ctx: Context, sk: torch.Tensor, msgs: torch.Tensor, seed: int,
                         stream=None) -> torch.Tensor:
    """Encryption with its randomness drawn from a seed: ct [Q][d][2][L][N]."""
    Q, d = msgs.shape
    ct = torch.empty((Q, d, 2, ctx.L, ctx.N), dtype=torch.uint64, device=msgs.device)
    nat.sanns_encrypt_query_seeded(ctx.handle, _ptr(sk), _ptr(msgs), Q, d, seed, _ptr(ct),
                                   _stream(stream))
    return ct


def public_key(ctx: Context, sk: torch.Tensor, seed: int, stream=None) -> torch.Tensor:
    """The client's public key [2][L][N] (sanns_public_key)."""
    pk = torch.empty((2, ctx.L, ctx.N), dtype=torch.uint64, device=sk.device)
    nat.sanns_public_key(ctx.handle, _ptr(sk), seed, _ptr(pk), _stream(stream))
    return pk


def decrypt_shares(ctx: Context, sk: torch.Tensor, ct: torch.Tensor,
                   qnorm2: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Client shares [M][N] uint32 of M ciphertexts [M][2][L][N]."""
    M = ct.shape[0]
    out = torch.empty((M, ctx.N), dtype=torch.uint32, device=ct.device)
    nat.sanns_decrypt_shares(ctx.handle, _ptr(sk), _ptr(ct), M, _ptr(qnorm2), _ptr(out),
                             _stream(stream))
    return out


class Distances:
    """Output and workspace buffers of sanns_distances for a fixed (Q, M)."""

    def __init__(self, ctx: Context, db: Database, Q: int,
                 work: Optional[np.ndarray] = None, mode: int = nat.SANNS_MODE_FUSED,
                 workspace: Optional[torch.Tensor] = None,
                 out_buffers: Optional[tuple] = None, private: bool = False):
        """workspace: optional uint8 device tensor of at least the required
        size, reused instead of a fresh allocation; out_buffers: optional
        pair of uint8 device tensors that hold the ciphertext outputs and the
        shares (at least M 2 L N 8 and M N 4 bytes), likewise reused;
        private: size the workspace for the circuit-private form
        (sanns_distances_cp; run() then needs the public keys)."""
        self.ctx, self.db, self.Q, self.mode = ctx, db, Q, mode
        self.private = private
        self.work = None if work is None else np.ascontiguousarray(work, dtype=np.uint32)
        self.M = Q * db.n_chunks if work is None else len(self.work)
        dev = db.mem.device
        size = nat.sanns_distances_cp_workspace if private else nat.sanns_distances_workspace
        self.ws_bytes = size(ctx.handle, db.desc, Q, self.M, mode)
        if workspace is not None and workspace.numel() >= self.ws_bytes:
            self.ws = workspace[:self.ws_bytes]
        else:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        shape_out, shape_share = (self.M, 2, ctx.L, ctx.N), (self.M, ctx.N)
        if out_buffers is not None:
            nb_out, nb_share = self.M * 2 * ctx.L * ctx.N * 8, self.M * ctx.N * 4
            if out_buffers[0].numel() < nb_out or out_buffers[1].numel() < nb_share:
                raise ValueError("output buffers are too small")
            self.ct_out = out_buffers[0][:nb_out].view(torch.uint64).view(shape_out)
            self.share = out_buffers[1][:nb_share].view(torch.uint32).view(shape_share)
        else:
            self.ct_out = torch.empty(shape_out, dtype=torch.uint64, device=dev)
            self.share = torch.empty(shape_share, dtype=torch.uint32, device=dev)

    def run(self, ct_in: torch.Tensor, mask_key: bytes, query_ids: torch.Tensor,
            stream=None, pk: Optional[torch.Tensor] = None, flood_bits: int = 0):
        """pk: [Q][2][L][N] public keys for the circuit-private form (the
        object must have been built with private=True)."""
        if ct_in.shape[0] != self.Q:
            raise ValueError("query count differs from the one the buffers were sized for")
        if (pk is not None) != self.private:
            raise ValueError("public keys are needed exactly when private=True")
        if pk is not None:
            nat.sanns_distances_cp(self.ctx.handle, self.db.desc, _ptr(ct_in), self.Q, mask_key,
                                   _ptr(query_ids), _ptr(pk), flood_bits, self.work, self.M,
                                   self.mode, _ptr(self.ct_out), _ptr(self.share),
                                   _ptr(self.ws), self.ws_bytes, _stream(stream))
        else:
            nat.sanns_distances(self.ctx.handle, self.db.desc, _ptr(ct_in), self.Q, mask_key,
                                _ptr(query_ids), self.work, self.M, self.mode,
                                _ptr(self.ct_out), _ptr(self.share), _ptr(self.ws),
                                self.ws_bytes, _stream(stream))
        return self.ct_out, self.share


def gathered_distances(ctx: Context, points: torch.Tensor, slot_point, row_query: np.ndarray,
                       ct_in: torch.Tensor, mask_key: bytes, query_ids: torch.Tensor,
                       norm_shares: Optional[torch.Tensor] = None,
                       tail: Optional[Database] = None,
                       workspace: Optional[torch.Tensor] = None, stream=None):
    """sanns_distances_gathered: chunk m holds points slot_point[m N:(m+1) N]
    (-1 padding) and belongs to query row_query[m]; with a tail database,
    every query also scans its chunks (rows M + q Ct + k).  points: device
    [n][d] uint8 / int8 points, or int32 / uint32 shares in [0, t) (then
    norm_shares [n] is required).  Returns (ct_out [rows][2][L][N], shares
    [rows][N])."""
    if points.dtype == torch.uint8:
        dtype = nat.SANNS_U8
    elif points.dtype == torch.int8:
        dtype = nat.SANNS_I8
    elif points.dtype in (torch.int32, torch.uint32):
        dtype = nat.SANNS_SHARE32
    else:
        raise ValueError("points must be uint8, int8 or 32-bit shares")
    n, d = points.shape
    rq = np.ascontiguousarray(row_query, dtype=np.uint32)
    M = len(rq)
    dev = points.device
    sp = slot_point if isinstance(slot_point, torch.Tensor) else torch.as_tensor(
        np.ascontiguousarray(slot_point, dtype=np.int64)).to(dev)
    if sp.numel() != M * ctx.N:
        raise ValueError("slot map must hold M N entries")
    Q = ct_in.shape[0]
    tdesc = None if tail is None else tail.desc
    rows = M + (0 if tail is None else Q * tail.n_chunks)
    ws_bytes = nat.sanns_distances_gathered_workspace(ctx.handle, d, Q, M, tdesc)
    ws = workspace[:ws_bytes] if workspace is not None and workspace.numel() >= ws_bytes \
        else torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ct_out = torch.empty((rows, 2, ctx.L, ctx.N), dtype=torch.uint64, device=dev)
    share = torch.empty((rows, ctx.N), dtype=torch.uint32, device=dev)
    nat.sanns_distances_gathered(ctx.handle, _ptr(points), dtype, n, d, _ptr(norm_shares),
                                 _ptr(sp.contiguous()), rq, M, tdesc, _ptr(ct_in), Q,
                                 mask_key, _ptr(query_ids), _ptr(ct_out), _ptr(share), _ptr(ws),
                                 ws_bytes, _stream(stream))
    return ct_out, share


def distances(ctx: Context, db: Database, ct_in: torch.Tensor, mask_key: bytes,
              query_ids: torch.Tensor, work: Optional[np.ndarray] = None,
              mode: int = nat.SANNS_MODE_FUSED, stream=None):
    """One-shot sanns_distances: returns (ct_out [M][2][L][N], shares [M][N])."""
    D = Distances(ctx, db, ct_in.shape[0], work, mode)
    return D.run(ct_in, mask_key, query_ids, stream)
