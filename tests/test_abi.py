"""CPU checks of the C-ABI library: it loads, exports every symbol include/pmr.h declares,
and validates configurations on the host (no device calls)."""
import ctypes
import re

import numpy as np
import pytest

from paper_1805_02247_amd import _lib as L
from paper_1805_02247_amd import api


def _declared():
    src = open(L.HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pmr_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_status_strings():
    lib = L.lib()
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert lib.pmr_status_string(st)


@pytest.mark.parametrize("bad", [
    dict(n_part=24), dict(n_part=8), dict(n_mesh=64, n_part=16), dict(n_out=64),
    dict(batch=0), dict(n_steps=0), dict(mlp_hidden=12), dict(box=0.0), dict(a1=0.05),
    dict(ckpt_every=-1), dict(precision=7), dict(loss_kind=3), dict(ic_order=3),
    dict(ic_order=-1), dict(halo_model=2), dict(halo_model=1, loss_kind=0),
    dict(halo_model=1, precision=1), dict(n_part=512, n_mesh=512,
                                                                     n_out=512, batch=32)])
def test_invalid_configs_rejected(bad):
    cfg = api.Config(**{**dict(n_part=16, n_mesh=16, n_out=16), **bad})
    assert api.workspace_bytes(cfg) == 0
    ctx = ctypes.c_void_p()
    c = cfg.c()
    assert L.lib().pmr_create(ctypes.byref(c), ctypes.c_void_p(256), 1 << 40, None,
                              ctypes.byref(ctx)) != 0


def test_workspace_plan_and_checks():
    cfg = api.Config(batch=2, n_part=16, n_mesh=32, n_out=16, n_steps=3, mlp_hidden=8)
    n = api.workspace_bytes(cfg)
    assert n > 0 and n % 256 == 0
    ctx = ctypes.c_void_p()
    c = cfg.c()
    lib = L.lib()
    # misaligned or short workspace
    assert lib.pmr_create(ctypes.byref(c), ctypes.c_void_p(256 + 8), n, None, ctypes.byref(ctx)) == -3
    assert lib.pmr_create(ctypes.byref(c), ctypes.c_void_p(256), n - 1, None, ctypes.byref(ctx)) == -3
    # checkpointing needs less memory than keeping every step
    more = api.workspace_bytes(api.Config(batch=1, n_part=32, n_mesh=32, n_out=32, n_steps=10))
    less = api.workspace_bytes(api.Config(batch=1, n_part=32, n_mesh=32, n_out=32, n_steps=10,
                                          ckpt_every=2))
    assert less < more
    # second-order initial conditions keep phi_ab, their adjoints and Psi2: 15 fields more
    lpt2 = api.workspace_bytes(api.Config(batch=1, n_part=32, n_mesh=32, n_out=32, n_steps=10,
                                          ic_order=2))
    assert lpt2 - more == 15 * 4 * 32 ** 3
    assert api.workspace_bytes(api.Config(batch=1, n_part=32, n_mesh=32, n_out=32, n_steps=10,
                                          ic_order=0)) == more
    # the two-network model keeps its weights and the 81 position-network input adjoints
    two = api.workspace_bytes(api.Config(batch=1, n_part=32, n_mesh=32, n_out=32, n_steps=10,
                                         halo_model=1, mlp_hidden=12))
    assert two > more + 81 * 4 * 32 ** 3


def test_primitives_reject_bad_shapes_without_touching_memory():
    lib = L.lib()
    assert lib.pmr_fft_r2c(24, 1, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == -2
    assert lib.pmr_fft_c2r(16, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == -1
    assert lib.pmr_sort_scratch_bytes(1000, 24, 1) == 0
    assert lib.pmr_cic_sort(16, 16, 1, 1.0, None, None, None, None, None, 0, None) == -1


def test_fft_tile_shape_validation():
    """Tile shapes are host state: valid ones are stored and read back per pass, invalid ones
    (pass, columns, threads, LDS size, points per thread, staging) are refused unchanged."""
    lib = L.lib()
    c, t, s = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()

    def get(n, p):
        assert lib.pmr_fft_get_tile(n, p, ctypes.byref(c), ctypes.byref(t), ctypes.byref(s)) == 0
        return (c.value, t.value, s.value)
    saved = {p: get(128, p) for p in (0, 1)}
    try:
        assert lib.pmr_fft_set_tile(128, 0, 32, 256, 2) == 0
        assert get(128, 0) == (32, 256, 2)
        assert lib.pmr_fft_set_tile(128, 0, 32, 256, 1) == 0
        assert lib.pmr_fft_set_tile(128, 1, 8, 512, 0) == 0
        assert get(128, 0) == (32, 256, 1) and get(128, 1) == (8, 512, 0)
        for bad in [(128, 3, 16, 256, 0), (128, 0, 12, 256, 0), (128, 0, 16, 384, 0),
                    (128, 1, 32, 256, 3), (128, 1, 32, 256, -1), (512, 0, 32, 256, 0),
                    (96, 0, 16, 256, 0), (16, 1, 8, 256, 0)]:
            assert lib.pmr_fft_set_tile(*bad) == -1, bad
        assert get(128, 0) == (32, 256, 1) and get(128, 1) == (8, 512, 0)
        assert lib.pmr_fft_get_tile(24, 0, ctypes.byref(c), ctypes.byref(t), ctypes.byref(s)) == -1
        assert lib.pmr_fft_get_tile(64, 3, ctypes.byref(c), ctypes.byref(t), ctypes.byref(s)) == -1
    finally:
        for p, v in saved.items():
            lib.pmr_fft_set_tile(128, p, *v)


def test_reconstruction_calls_validate_arguments_on_the_host():
    """Bad arguments of the driver calls are refused before any device work."""
    lib = L.lib()
    P = ctypes.c_void_p
    fake = P(4096)  # never dereferenced: every call below fails validation first
    order = (ctypes.c_int * 3)(0, 1, 1)
    assert lib.pmr_vec_work_bytes(1000, -1) == 0
    assert lib.pmr_vec_work_bytes(1000, 4) > lib.pmr_vec_work_bytes(1000, 0) > 0
    assert lib.pmr_vec_dot(0, fake, fake, fake, fake, None) == -1
    assert lib.pmr_vec_dot(10, None, fake, fake, fake, None) == -1
    assert lib.pmr_vec_axpby(10, 1.0, fake, 1.0, fake, None, None) == -1
    # count > m, duplicate slot, slot out of range, g aliasing d, m out of range
    assert lib.pmr_lbfgs_direction(10, 2, 3, order, fake, fake, fake, fake, P(8192), fake,
                                   fake, None) == -1
    assert lib.pmr_lbfgs_direction(10, 4, 3, order, fake, fake, fake, fake, P(8192), fake,
                                   fake, None) == -1
    bad = (ctypes.c_int * 1)(5)
    assert lib.pmr_lbfgs_direction(10, 4, 1, bad, fake, fake, fake, fake, P(8192), fake,
                                   fake, None) == -1
    assert lib.pmr_lbfgs_direction(10, 4, 0, None, None, None, None, None, fake, fake, fake,
                                   None) == -1
    assert lib.pmr_lbfgs_direction(10, 65, 0, None, None, None, None, None, P(8192), fake,
                                   fake, None) == -1
    assert lib.pmr_power_work_bytes(0) == 0 and lib.pmr_power_work_bytes(8) > 0
    need = lib.pmr_power_work_bytes(8)
    assert lib.pmr_power_bins(12, 100.0, fake, fake, 8, fake, fake, need, None) == -2
    assert lib.pmr_power_bins(16, 100.0, fake, fake, 33, fake, fake, need, None) == -2
    assert lib.pmr_power_bins(16, 0.0, fake, fake, 8, fake, fake, need, None) == -1
    assert lib.pmr_power_bins(16, 100.0, fake, fake, 8, fake, fake, need - 8, None) == -3


def test_device_lbfgs_validates_arguments_on_the_host():
    """The device-driven optimiser's calls refuse bad parameters and pointers before any
    device work."""
    lib = L.lib()
    P = ctypes.c_void_p
    f = [P(4096 * (k + 1)) for k in range(12)]  # distinct, never dereferenced
    assert lib.pmr_lbfgs_state_bytes(0) == 0
    assert lib.pmr_lbfgs_state_bytes(10) == ctypes.sizeof(L.PmrLbfgsState) + 11 * 16

    def params(**kw):
        p = dict(m=10, max_iter=20, max_halvings=30, c1=1e-4, curvature_eps=1e-10,
                 rel_tol=1e-3, stop_below=float("-inf"))
        p.update(kw)
        return L.PmrLbfgsParams(**p)

    for bad in (dict(m=0), dict(m=65), dict(max_iter=0), dict(max_halvings=-1), dict(c1=0.0),
                dict(c1=1.0), dict(rel_tol=-1.0), dict(stop_below=float("nan")),
                dict(curvature_eps=float("nan"))):
        assert lib.pmr_lbfgs_init(100, ctypes.byref(params(**bad)), *f[:10]) == -1, bad
    assert lib.pmr_lbfgs_init(100, None, *f[:10]) == -1
    assert lib.pmr_lbfgs_init(0, ctypes.byref(params()), *f[:10]) == -1
    g_is_d = [f[0], f[1], f[2], f[2]] + f[4:10]
    assert lib.pmr_lbfgs_init(100, ctypes.byref(params()), *g_is_d) == -1
    assert lib.pmr_lbfgs_trial(100, f[0], f[1], f[2], f[1], None) == -1  # xt aliases x
    assert lib.pmr_lbfgs_trial(100, None, f[1], f[2], f[3], None) == -1
    upd = f[:12]
    assert lib.pmr_lbfgs_update(100, 0, *upd, None) == -1
    assert lib.pmr_lbfgs_update(100, 65, *upd, None) == -1
    alias = list(upd)
    alias[4] = alias[2]  # xt aliases x
    assert lib.pmr_lbfgs_update(100, 4, *alias, None) == -1


def test_lbfgs_state_layout_matches_the_header(tmp_path):
    """The ctypes view of pmr_lbfgs_state and pmr_lbfgs_params has the C layout of the
    header (compiled with the host C compiler)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    names = [n for n, _ in L.PmrLbfgsState._fields_]
    pnames = [n for n, _ in L.PmrLbfgsParams._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof(pmr_lbfgs_state, {n}));\n' for n in names)
    body += "".join(f'  printf("%zu\\n", offsetof(pmr_lbfgs_params, {n}));\n' for n in pnames)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "pmr.h"\nint main(void) {\n'
                   '  printf("%zu\\n%zu\\n", sizeof(pmr_lbfgs_state), sizeof(pmr_lbfgs_params));\n'
                   + body + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    inc = str(__import__("os").path.dirname(L.HEADER_PATH))
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(L.PmrLbfgsState), ctypes.sizeof(L.PmrLbfgsParams)]
    want += [getattr(L.PmrLbfgsState, n).offset for n in names]
    want += [getattr(L.PmrLbfgsParams, n).offset for n in pnames]
    assert got == want
