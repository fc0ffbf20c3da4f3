"""GPU parity of the 3-D real FFTs (pmr_fft_r2c / pmr_fft_c2r) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import mesh as M
from paper_1805_02247_amd import api
from _gpu import DEV, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu

TOL = 2e-6  # FP32 FFT, rel-L2 over the whole spectrum (n <= 512)


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_r2c_matches_oracle(n):
    require_gpu()
    say(f"r2c n={n}")
    x = synth.unit_normal(n, (2, n, n, n)).astype(np.float32)
    X = api.fft_r2c(torch.from_numpy(x).to(DEV)).cpu().numpy()
    for b in range(2):
        ref = M.rfft3(x[b].astype(np.float64))
        e = rel_l2(X[b], ref)
        say(f"  item {b}: rel-L2 {e:.2e}")
        assert e < TOL


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_c2r_matches_oracle(n):
    require_gpu()
    say(f"c2r n={n}")
    x = synth.unit_normal(n + 1, (2, n, n, n))
    X = np.stack([M.rfft3(x[b]) for b in range(2)]).astype(np.complex64)
    y = api.fft_c2r(torch.from_numpy(X).to(DEV)).cpu().numpy()
    for b in range(2):
        ref = M.irfft3(X[b].astype(np.complex128), n)
        e = rel_l2(y[b], ref)
        say(f"  item {b}: rel-L2 {e:.2e}")
        assert e < TOL


def test_c2r_ignores_what_a_real_field_cannot_carry():
    """Arbitrary (non-Hermitian) input: same result as the oracle's inverse (irfftn)."""
    require_gpu()
    n = 32
    X = synth.random_modes_direction(4, n).astype(np.complex64)[None]
    y = api.fft_c2r(torch.from_numpy(X).to(DEV)).cpu().numpy()[0]
    ref = M.irfft3(X[0].astype(np.complex128), n)
    e = rel_l2(y, ref)
    say(f"non-Hermitian c2r rel-L2 {e:.2e}")
    assert e < TOL


def _separable(n, seed):
    v = synth.unit_normal(seed, (6, n))
    x = (v[0][:, None, None] * v[1][None, :, None] * v[2][None, None, :]
         + v[3][:, None, None] * v[4][None, :, None] * v[5][None, None, :])
    return v, x.astype(np.float32)


@pytest.mark.parametrize("n,staging", [(256, None), (512, None), (512, 2)])
def test_r2c_large_separable(n, staging):
    """At full size: a sum of two separable fields, whose transform is the sum of outer
    products of 1-D transforms; checked on 8 sampled kx planes. With the tuned tiles, and at
    512 also with both strided passes on LDS-staged radix-4 stages."""
    require_gpu()
    import paper_1805_02247_amd as P
    say(f"r2c separable n={n} staging={staging}")
    v, x = _separable(n, 7)
    saved = {p: P.fft_get_tile(n, p) for p in (P.PMR_FFT_YPASS, P.PMR_FFT_XPASS)}
    try:
        if staging is not None:
            for p in saved:
                P.fft_set_tile(n, p, 16, 512, staging)
        X = api.fft_r2c(torch.from_numpy(x).to(DEV)[None])[0]
    finally:
        for p, t in saved.items():
            P.fft_set_tile(n, p, *t)
    del x
    planes = np.random.default_rng(n).choice(n, 8, replace=False)
    # closed form from the FP64 factors; the float32 rounding of the input adds ~1e-7
    F = [np.fft.fft(v[i]) for i in range(6)]
    Fz = [np.fft.rfft(v[i]) for i in (2, 5)]
    got = np.stack([X[ix].cpu().numpy() for ix in planes])
    ref = np.stack([F[0][ix] * F[1][:, None] * Fz[0][None, :] + F[3][ix] * F[4][:, None] * Fz[1][None, :]
                    for ix in planes])
    e = rel_l2(got, ref)
    say(f"  8 planes: rel-L2 {e:.2e}")
    assert e < TOL


@pytest.mark.parametrize("n", [256, 512])
def test_roundtrip_large(n):
    require_gpu()
    say(f"round trip n={n}")
    _, x = _separable(n, 9)
    xt = torch.from_numpy(x).to(DEV)[None]
    y = api.fft_c2r(api.fft_r2c(xt))
    e = (torch.linalg.vector_norm((y - xt).double()) / torch.linalg.vector_norm(xt.double())).item()
    say(f"  rel-L2 {e:.2e}")
    assert e < 2 * TOL


SHAPES = [(8, 256), (16, 256), (32, 256), (8, 512), (16, 512), (32, 512)]


@pytest.mark.parametrize("n", [64, 128])
def test_every_tile_shape_and_staging(n):
    """Each supported tile shape, with register staging and LDS staging of radix-8 and of
    radix-4 stages, in each strided pass, against the oracle (the other pass held at its
    current shape)."""
    require_gpu()
    import paper_1805_02247_amd as P
    from paper_1805_02247_amd.tune import candidates
    saved = {p: P.fft_get_tile(n, p) for p in (P.PMR_FFT_YPASS, P.PMR_FFT_XPASS)}
    x = synth.unit_normal(3 * n, (1, n, n, n)).astype(np.float32)
    ref = M.rfft3(x[0].astype(np.float64))
    X = np.stack([ref]).astype(np.complex64)
    ref_inv = M.irfft3(X[0].astype(np.complex128), n)
    try:
        for p in saved:
            for c in candidates(n):
                P.fft_set_tile(n, p, *c)
                got = api.fft_r2c(torch.from_numpy(x).to(DEV)).cpu().numpy()[0]
                inv = api.fft_c2r(torch.from_numpy(X).to(DEV)).cpu().numpy()[0]
                e1, e2 = rel_l2(got, ref), rel_l2(inv, ref_inv)
                say(f"  n={n} pass {p} {c}: r2c {e1:.2e} c2r {e2:.2e}")
                assert e1 < TOL and e2 < TOL
            P.fft_set_tile(n, p, *saved[p])
    finally:
        for p, v in saved.items():
            P.fft_set_tile(n, p, *v)
