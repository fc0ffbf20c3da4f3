"""pmr_lbfgs_direction_noalloc (the L-BFGS direction with its scratch in a fixed array inside
the library) against pmr_lbfgs_direction with a caller-owned work buffer: bit for bit, on
two calls in a row, the second with a smaller vector and history; and its argument checks."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1805_02247_amd import _lib as L
from paper_1805_02247_amd.api import _ptr, _stream
from _gpu import DEV, require_gpu, say

pytestmark = pytest.mark.gpu


def _case(n, m, order, seed):
    g = torch.Generator().manual_seed(seed)
    S = torch.randn(m, n, generator=g)
    Y = (S + 0.3 * torch.randn(m, n, generator=g)).to(DEV)
    S = S.to(DEV)
    grad = torch.randn(n, generator=g).to(DEV)
    sy = (S.double() * Y.double()).sum(1).contiguous()
    yy = (Y.double() * Y.double()).sum(1).contiguous()
    return S, Y, grad, sy, yy, (ctypes.c_int * max(len(order), 1))(*order)


def _with_work(n, m, order, S, Y, g, sy, yy, arr):
    d = torch.empty(n, device=DEV)
    work = torch.empty(int(L.lib().pmr_vec_work_bytes(n, m)), dtype=torch.uint8, device=DEV)
    L.check(L.lib().pmr_lbfgs_direction(n, m, len(order), arr, _ptr(S), _ptr(Y), _ptr(sy),
                                        _ptr(yy), _ptr(g), _ptr(d), _ptr(work), _stream()))
    return d


def _noalloc(n, m, order, S, Y, g, sy, yy, arr):
    d = torch.empty(n, device=DEV)
    L.check(L.lib().pmr_lbfgs_direction_noalloc(n, m, len(order), arr, _ptr(S), _ptr(Y),
                                                _ptr(sy), _ptr(yy), _ptr(g), _ptr(d),
                                                _stream()))
    return d


def test_noalloc_direction_equals_work_buffer_version():
    require_gpu()
    # large first (every partial-sum slot in use), then smaller vector and history
    for n, m, order, seed in ((3 * (1 << 20) + 77, 10, [4, 3, 2, 1, 0, 9, 8], 1),
                              (5000, 4, [1, 0, 3], 2)):
        say(f"noalloc: n={n}, m={m}, history {order}")
        S, Y, g, sy, yy, arr = _case(n, m, order, seed)
        a = _noalloc(n, m, order, S, Y, g, sy, yy, arr)
        b = _with_work(n, m, order, S, Y, g, sy, yy, arr)
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)
    # an empty history gives d = -g exactly
    S, Y, g, sy, yy, arr = _case(1000, 2, [], 3)
    assert torch.equal(_noalloc(1000, 2, [], S, Y, g, sy, yy, arr), -g)


def test_noalloc_direction_argument_checks():
    require_gpu()
    S, Y, g, sy, yy, arr = _case(100, 2, [0], 4)
    d = torch.empty(100, device=DEV)
    lib = L.lib()
    big = (ctypes.c_int * 1)(0)
    # history beyond the fixed array, repeated slot, aliasing g and d, n = 0
    assert lib.pmr_lbfgs_direction_noalloc(100, 65, 1, big, _ptr(S), _ptr(Y), _ptr(sy),
                                           _ptr(yy), _ptr(g), _ptr(d), _stream()) == -2
    rep = (ctypes.c_int * 2)(0, 0)
    assert lib.pmr_lbfgs_direction_noalloc(100, 2, 2, rep, _ptr(S), _ptr(Y), _ptr(sy),
                                           _ptr(yy), _ptr(g), _ptr(d), _stream()) == -1
    assert lib.pmr_lbfgs_direction_noalloc(100, 2, 1, arr, _ptr(S), _ptr(Y), _ptr(sy),
                                           _ptr(yy), _ptr(g), _ptr(g), _stream()) == -1
    assert lib.pmr_lbfgs_direction_noalloc(0, 2, 1, arr, _ptr(S), _ptr(Y), _ptr(sy),
                                           _ptr(yy), _ptr(g), _ptr(d), _stream()) == -1
