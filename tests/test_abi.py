"""CPU checks of the C ABI: the library loads, exports every declared symbol,
derives the same parameters as the oracle, and rejects bad arguments on the
host before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1904_02033_amd import native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "sanns.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sanns_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = nat.load()
    names = _header_functions()
    assert set(names) == set(nat.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,L,bits", [(16, 1, 8), (4096, 2, 25), (8192, 3, 25),
                                      (8192, 3, 26), (16384, 4, 30)])
def test_params_derive_matches_oracle(N, L, bits):
    p = nat.sanns_params_derive(N, L, bits)
    assert [p.q[l] for l in range(L)] == oracle.rns_primes(N, L)
    assert p.t == oracle.plain_modulus(N, bits)
    assert p.N == N and p.L == L


def _status(fn, *args):
    return fn(*args)


def test_host_argument_errors():
    lib = nat.load()
    p = nat.sanns_params()
    assert lib.sanns_params_derive(1000, 2, 25, ctypes.byref(p)) == nat.SANNS_E_INVALID
    assert lib.sanns_params_derive(4096, 5, 25, ctypes.byref(p)) == nat.SANNS_E_INVALID
    assert lib.sanns_params_derive(4096, 2, 40, ctypes.byref(p)) == nat.SANNS_E_INVALID
    assert lib.sanns_params_derive(4096, 2, 25, None) == nat.SANNS_E_INVALID
    h = ctypes.c_void_p()
    # parameter checks run before any device call
    good = nat.sanns_params_derive(4096, 2, 25)
    bad = nat.sanns_params_derive(4096, 2, 25)
    bad.q[1] = bad.q[0]
    assert lib.sanns_ctx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == nat.SANNS_E_PARAMS
    assert b"repeats" in lib.sanns_last_error()
    bad = nat.sanns_params_derive(4096, 2, 25)
    bad.q[0] += 2 * 4096  # = 1 mod 2N but composite or not -- check primality path
    st = lib.sanns_ctx_create(ctypes.byref(bad), 0, ctypes.byref(h))
    if oracle.is_prime(bad.q[0]):
        assert st in (nat.SANNS_E_PARAMS, nat.SANNS_E_DEVICE)
    else:
        assert st == nat.SANNS_E_PARAMS
    bad = nat.sanns_params_derive(4096, 2, 25)
    bad.q[0] += 2  # not 1 mod 2N
    assert lib.sanns_ctx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == nat.SANNS_E_PARAMS
    # 128-bit security cap: three 54-bit primes at N = 4096 exceed 109 bits
    bad = nat.sanns_params_derive(4096, 3, 25)
    assert lib.sanns_ctx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == nat.SANNS_E_PARAMS
    assert b"cap" in lib.sanns_last_error()
    small = nat.sanns_params_derive(16, 2, 10)
    assert lib.sanns_ctx_create(ctypes.byref(small), 0, ctypes.byref(h)) == nat.SANNS_E_PARAMS
    bad = nat.sanns_params_derive(4096, 2, 25)
    bad.t = 1 << 31
    assert lib.sanns_ctx_create(ctypes.byref(bad), 0, ctypes.byref(h)) == nat.SANNS_E_PARAMS
    assert lib.sanns_ctx_create(None, 0, ctypes.byref(h)) == nat.SANNS_E_INVALID
    # null contexts / buffers
    assert lib.sanns_encode_db(None, None, 0, 1, None, None, None) == nat.SANNS_E_INVALID
    assert lib.sanns_distances(None, None, None, 1, None, None, None, 0, 0, None, None, None,
                               0, None) == nat.SANNS_E_INVALID
    assert lib.sanns_decrypt_shares(None, None, None, 1, None, None, None) == \
        nat.SANNS_E_INVALID
    assert lib.sanns_encrypt_query(None, None, None, 1, 1, None, None, None, None) == \
        nat.SANNS_E_INVALID
    assert lib.sanns_set_schedule(None, 0, 1, 4) == nat.SANNS_E_INVALID
    assert lib.sanns_device_status(None, None) == nat.SANNS_E_INVALID
    lib.sanns_ctx_destroy(None)
