"""Device arithmetic that bitwise parity rests on, probed directly on the
GPU: the library's Philox4x32-10 against the oracle's, its small-angle
sin/cos polynomial against the oracle's, and the binary64 square root,
division and rint (ties to even) against IEEE 754 as numpy computes them on
the host, on 10^7 random operands."""
import ctypes
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libdevice_probe.so")


@pytest.fixture(scope="module")
def probe():
    # initialise the GPU through PyTorch first, as the library's own users do,
    # so that one HIP runtime serves the process
    import torch
    assert torch.cuda.is_available(), "the device probe needs a GPU"
    torch.cuda.init()
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is missing: build with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    U, D = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)
    lib.probe_philox.argtypes = [U, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, U]
    lib.probe_f64.argtypes = [D, D, ctypes.c_int64, D, D, D]
    lib.probe_sincos.argtypes = [D, ctypes.c_int64, D, D]
    return lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def test_philox_matches_the_oracle(probe):
    """10^7 random counters under two keys, every output word compared."""
    rng = np.random.Generator(np.random.PCG64(91))
    n = 5 * 10 ** 6
    for k0, k1 in ((0x9E3779B9, 0x01234567), (0xFFFFFFFF, 0x00000000)):
        ctr = np.ascontiguousarray(rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32))
        out = np.zeros_like(ctr)
        assert probe.probe_philox(_p(ctr, ctypes.c_uint32), n, k0, k1, _p(out, ctypes.c_uint32)) == 0
        want = oracle.philox4x32_10_many(ctr, (k0, k1))
        bad = np.argwhere(np.any(out != want, axis=1))
        assert bad.size == 0, bad[:5]


def test_sqrt_division_rint_are_ieee(probe):
    rng = np.random.Generator(np.random.PCG64(92))
    n = 10 ** 7
    a = np.ascontiguousarray(np.exp(rng.uniform(-700, 700, size=n)))
    b = rng.uniform(-1e6, 1e6, size=n)
    b[: n // 10] = np.floor(b[: n // 10]) + 0.5  # exact ties for rint
    b = np.ascontiguousarray(b)
    sq, dv, ri = (np.zeros(n) for _ in range(3))
    D = ctypes.c_double
    assert probe.probe_f64(_p(a, D), _p(b, D), n, _p(sq, D), _p(dv, D), _p(ri, D)) == 0
    assert np.array_equal(sq.view(np.uint64), np.sqrt(a).view(np.uint64))
    assert np.array_equal(dv.view(np.uint64), (a / b).view(np.uint64))
    assert np.array_equal(ri, np.rint(b))


def test_small_angle_sincos_matches_the_oracle(probe):
    rng = np.random.Generator(np.random.PCG64(93))
    n = 20000
    d = np.ascontiguousarray(rng.uniform(-0.2, 0.2, size=n))
    c, s = np.zeros(n), np.zeros(n)
    D = ctypes.c_double
    assert probe.probe_sincos(_p(d, D), n, _p(c, D), _p(s, D)) == 0
    for i in range(n):
        assert (c[i], s[i]) == oracle.sincos(d[i]), i
