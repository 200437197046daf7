"""C-ABI checks that need no GPU: library loads, exports every declared symbol,
validates arguments before any HIP call, and its host-side plan tables (space-time
kernel, block-shift schedule) agree with the oracle."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1809_04195_amd as T
from oracle import t2s as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(T.LIB_PATH), reason="libt2s.so not built")


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "t2s.h")).read()
    return sorted(set(re.findall(r"\b(t2s_\w+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (t2s_\w+)", out))
    declared = header_symbols()
    assert declared, "no declarations parsed"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    # the binding wraps every declared entry point
    assert set(declared) <= set(T.EXPORTED)
    assert T.t2s_version() >= 100


def _classes(ny=32, nz=48, C=2, S=1, T_=6, seed=0):
    rng = np.random.default_rng(seed)
    masks = (rng.random((T_, ny, nz)) < 0.3).astype(np.uint8)
    return [(ny, nz, C, S, masks)], masks


def _phi(T_=6, K=3):
    q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((T_, K)))
    return q.astype(np.float32)


def _create(phi, cls, **kw):
    p = T.make_params(phi, kw.pop("lam", 0.01), kw.pop("rho", 0.1), **kw)
    arr, keep = T.make_classes(cls)
    h = ctypes.c_void_p()
    code = T.lib().t2s_plan_create(ctypes.byref(p), arr, len(cls), ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("case,expected", [
    ("k_too_big", T.T2S_ESHAPE),
    ("k_gt_t", T.T2S_ESHAPE),
    ("odd_grid", T.T2S_ESHAPE),
    ("unsupported_len", T.T2S_EUNSUPPORTED),
    ("nan_phi", T.T2S_ENONFINITE),
    ("bad_block", T.T2S_EINVAL),
    ("bad_rho", T.T2S_EINVAL),
    ("bad_mask", T.T2S_EINVAL),
    ("zero_coils", T.T2S_ESHAPE),
    ("tol_without_window", T.T2S_EINVAL),
    ("bad_nmaps", T.T2S_ESHAPE),
    ("ny_not_a_column_length", T.T2S_ESHAPE),
])
def test_plan_create_rejects(case, expected):
    phi = _phi()
    cls, masks = _classes()
    kw = {}
    if case == "k_too_big":
        phi = np.ones((12, 9), np.float32)
        cls = [(32, 48, 2, 1, np.ones((12, 32, 48), np.uint8))]
    elif case == "k_gt_t":
        phi = np.ones((2, 3), np.float32)
        cls = [(32, 48, 2, 1, np.ones((2, 32, 48), np.uint8))]
    elif case == "odd_grid":
        cls = [(40, 48, 2, 1, np.ones((6, 40, 48), np.uint8))]
    elif case == "unsupported_len":
        cls = [(112, 48, 2, 1, np.ones((6, 112, 48), np.uint8))]
    elif case == "nan_phi":
        phi = phi.copy()
        phi[2, 1] = np.nan
    elif case == "bad_block":
        kw["block"] = 6
    elif case == "bad_rho":
        kw["rho"] = 0.0
    elif case == "bad_mask":
        m = masks.copy()
        m[0, 0, 0] = 3
        cls = [(32, 48, 2, 1, m)]
    elif case == "zero_coils":
        cls = [(32, 48, 0, 1, masks)]
    elif case == "tol_without_window":
        kw.update(tol=1e-4, freeze_window=0)
    elif case == "bad_nmaps":
        cls = [(32, 48, 2, 1, masks, 3)]
    elif case == "ny_not_a_column_length":
        cls = [(260, 48, 2, 1, np.ones((6, 260, 48), np.uint8))]
    code, h = _create(phi, cls, **kw)
    assert code == expected, (code, T.t2s_last_error())
    assert T.t2s_last_error()


def test_null_arguments():
    L = T.lib()
    h = ctypes.c_void_p()
    assert L.t2s_plan_create(None, None, 0, ctypes.byref(h)) == T.T2S_EINVAL
    assert L.t2s_plan_create(None, None, 0, None) == T.T2S_EINVAL
    assert L.t2s_reconstruct(None, 0, None) == T.T2S_EINVAL
    assert L.t2s_load_slices(None, 0, 0, 1, None, None, 0, None) == T.T2S_EINVAL


def test_plan_state_errors_without_gpu():
    phi = _phi()
    cls, masks = _classes()
    code, h = _create(phi, cls)
    assert code == 0
    L = T.lib()
    n = ctypes.c_size_t()
    assert L.t2s_plan_workspace_bytes(h, ctypes.byref(n)) == 0 and n.value > 0
    # not bound yet: state errors, before any HIP call
    buf = np.zeros(10, np.complex64)
    assert L.t2s_load_slices(h, 0, 0, 1, buf.ctypes.data, buf.ctypes.data, 0, None) == T.T2S_ESTATE
    assert L.t2s_reconstruct(h, 0, None) == T.T2S_ESTATE
    # bad binds
    assert L.t2s_plan_bind_workspace(h, None, n.value, None) == T.T2S_ENOMEM
    assert L.t2s_plan_bind_workspace(h, ctypes.c_void_p(4096), n.value - 1, None) == T.T2S_ENOMEM
    # bad slice range / class / enum
    assert L.t2s_load_slices(h, 1, 0, 1, buf.ctypes.data, buf.ctypes.data, 0, None) == T.T2S_EINVAL
    assert L.t2s_load_slices(h, 0, 0, 2, buf.ctypes.data, buf.ctypes.data, 0, None) == T.T2S_EINVAL
    assert L.t2s_reconstruct(h, 7, None) == T.T2S_EINVAL
    rep = T.t2s_slice_report()
    assert L.t2s_get_slice_report(h, 0, 0, ctypes.byref(rep)) == T.T2S_ESTATE
    assert L.t2s_plan_destroy(h) == 0


def test_fista_pre_and_post_step_validation_without_gpu():
    """Argument and state checks of the FISTA, readout pre-step and post-step entry
    points all run before any HIP call."""
    L = T.lib()
    buf = np.zeros(16, np.complex64)
    p = buf.ctypes.data
    # readout pre-step: shape checks first; an empty array needs no pointers
    assert L.t2s_readout_ifft(100, 2, 10, p, p + 8, None) == T.T2S_ESHAPE     # no FFT plan for 100
    assert L.t2s_readout_ifft(64, 0, 10, p, p + 8, None) == T.T2S_ESHAPE
    assert L.t2s_readout_ifft(64, 2, -1, p, p + 8, None) == T.T2S_ESHAPE
    assert L.t2s_readout_ifft(64, 2, 0, None, None, None) == 0
    assert L.t2s_readout_ifft(64, 2, 10, None, p, None) == T.T2S_EINVAL
    assert L.t2s_readout_ifft(64, 1, 1, p, p + 8, None) == T.T2S_EINVAL        # overlapping arrays
    phi = _phi()
    cls, _ = _classes()
    code, h = _create(phi, cls)
    assert code == 0
    f = ctypes.c_float
    # FISTA: mode, iteration count and step checked, then the state (nothing bound)
    assert L.t2s_fista(None, T.T2S_BATCHED, 5, f(0.5), None) == T.T2S_EINVAL
    assert L.t2s_fista(h, T.T2S_BATCHED_GRAPH, 5, f(0.5), None) == T.T2S_EINVAL
    assert L.t2s_fista(h, T.T2S_BATCHED, -1, f(0.5), None) == T.T2S_EINVAL
    assert L.t2s_fista(h, T.T2S_BATCHED, 5, f(0.0), None) == T.T2S_EINVAL
    assert L.t2s_fista(h, T.T2S_BATCHED, 5, f(float("inf")), None) == T.T2S_EINVAL
    assert L.t2s_fista(h, T.T2S_BATCHED, 5, f(0.5), None) == T.T2S_ESTATE
    Lv = np.zeros(1)
    dp = Lv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.t2s_lipschitz(h, 0, 0, dp, None) == T.T2S_EINVAL
    assert L.t2s_lipschitz(h, 1, 10, dp, None) == T.T2S_EINVAL                   # no class 1
    assert L.t2s_lipschitz(h, 0, 10, None, None) == T.T2S_EINVAL
    assert L.t2s_lipschitz(h, 0, 10, dp, None) == T.T2S_ESTATE
    # post-step
    assert L.t2s_wavelet_denoise(h, 0, 0, 1, 0, f(0.1), None) == T.T2S_EINVAL
    assert L.t2s_wavelet_denoise(h, 0, 0, 1, 5, f(0.1), None) == T.T2S_EINVAL
    assert L.t2s_wavelet_denoise(h, 0, 0, 1, 2, f(-1.0), None) == T.T2S_EINVAL
    assert L.t2s_wavelet_denoise(h, 0, 0, 2, 2, f(0.1), None) == T.T2S_EINVAL    # slices past the class
    assert L.t2s_wavelet_denoise(h, 0, 0, 1, 2, f(0.1), None) == T.T2S_ESTATE
    rows = np.zeros((9, 3), np.float32)
    rp = rows.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert L.t2s_backproject(h, 0, 0, 1, 9, rp, p, None) == T.T2S_EINVAL         # more than 8 echo times
    assert L.t2s_backproject(h, 0, 0, 1, 0, rp, p, None) == T.T2S_EINVAL
    assert L.t2s_backproject(h, 0, 0, 1, 2, None, p, None) == T.T2S_EINVAL
    rows[1, 2] = np.nan
    assert L.t2s_backproject(h, 0, 0, 1, 2, rp, p, None) == T.T2S_ENONFINITE
    rows[1, 2] = 0.0
    assert L.t2s_backproject(h, 0, 0, 1, 2, rp, p, None) == T.T2S_ESTATE
    assert L.t2s_plan_destroy(h) == 0


def test_schedule_and_order_validation():
    phi = _phi()
    cls, masks = _classes()
    code, h = _create(phi, cls)
    assert code == 0
    L = T.lib()
    assert T.t2s_get_order(h, 0) == 0      # 32 x 48: small Psi table, one LDS buffer
    assert L.t2s_set_order(h, 0, 16) == T.T2S_EINVAL
    assert L.t2s_set_order(h, 1, 0) == T.T2S_EINVAL
    assert L.t2s_set_order(h, 0, T.T2S_ORDER_XCD_PASS_A | T.T2S_ORDER_XCD_PASS_C) == 0
    assert T.t2s_get_order(h, 0) == 3
    assert L.t2s_set_order(h, 0, T.T2S_ORDER_XCD_PASS_B | T.T2S_ORDER_PASS_C_LDS2) == 0
    assert T.t2s_get_order(h, 0) == 12
    assert L.t2s_set_schedule(h, 0, -1, 1) == T.T2S_EINVAL
    assert L.t2s_set_schedule(h, 0, 2, 9) == T.T2S_EINVAL
    assert L.t2s_set_schedule(h, 0, 2, 3) == 0
    assert T.t2s_get_schedule(h, 0) == (2, 3)
    T.t2s_plan_destroy(h)


@pytest.mark.parametrize("ny,nz,K,expected", [
    (384, 384, 5, 12),    # 9.4 MB Psi table: pass B coil-fastest; 384 points: two LDS buffers
    (256, 256, 4, 4),     # 3.1 MB table; one LDS buffer
    (64, 64, 3, 0),
])
def test_default_schedule_flags(ny, nz, K, expected):
    phi = _phi(T_=6, K=K)
    masks = np.zeros((6, ny, nz), np.uint8)
    masks[:, 0, 0] = 1
    code, h = _create(phi, [(ny, nz, 2, 1, masks)])
    assert code == 0
    assert T.t2s_get_order(h, 0) == expected
    T.t2s_plan_destroy(h)


def test_psi_table_matches_oracle():
    phi = _phi(T_=7, K=3)
    ny, nz = 32, 48
    masks = (np.random.default_rng(3).random((7, ny, nz)) < 0.4).astype(np.uint8)
    code, h = _create(phi, [(ny, nz, 2, 1, masks)])
    assert code == 0
    got = T.t2s_get_psi(h, 0, 3, ny, nz)                            # [tri][z'][y']
    psi = O.space_time_kernel(phi.astype(np.float64), masks.astype(bool))  # [K][K][y][z] centred
    tri = 0
    for k in range(3):
        for l in range(k, 3):
            ref = np.fft.ifftshift(psi[k, l]).T / (ny * nz)          # uncentred, transposed, / N
            assert np.allclose(got[tri], ref, rtol=1e-6, atol=1e-9), (k, l)
            tri += 1
    T.t2s_plan_destroy(h)


def test_block_shift_matches_oracle():
    for seed in (0, 1, 12345, 2**63 + 7):
        for g in (0, 1, 17, 319):
            for k in (0, 1, 2, 99, 499):
                for b in (4, 8, 16):
                    assert T.t2s_block_shift(seed, g, k, b) == O.block_shift(seed, g, k, b)


def test_set_initial_before_load_is_a_state_error():
    phi = _phi()
    cls, masks = _classes()
    code, h = _create(phi, cls)
    a0 = np.zeros((1, 3, 32, 48), np.complex64)
    assert T.lib().t2s_set_initial(h, 0, 0, 1, a0.ctypes.data, 0, None) == T.T2S_ESTATE
    T.t2s_plan_destroy(h)


def test_nonfinite_host_inputs_rejected_without_touching_the_gpu():
    # NaN / Inf in host inputs that are checked before any HIP call: the basis at plan
    # creation and the echo-time rows of the back-projection (slices with data need a
    # bound workspace, so their checks run in the GPU tests)
    cls, masks = _classes()
    for bad in (np.nan, np.inf):
        phi = _phi()
        phi[1, 0] = bad
        code, h = _create(phi, cls)
        assert code == T.T2S_ENONFINITE
    code, h = _create(_phi(), cls)
    assert code == 0
    ph = np.ones((2, 3), np.float32)
    ph[0, 2] = np.nan
    out = np.zeros(1, np.complex64)
    assert T.lib().t2s_backproject(h, 0, 0, 1, 2, ph.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), out.ctypes.data,
                                   None) == T.T2S_ENONFINITE
    T.t2s_plan_destroy(h)


def test_unet_create_validation_and_sizes():
    L = T.lib()
    h = ctypes.c_void_p()
    assert L.t2s_unet_create(0, 32, 4, 1, 256, 256, ctypes.byref(h)) == T.T2S_EINVAL
    assert L.t2s_unet_create(4, 32, 4, 1, 100, 256, ctypes.byref(h)) == T.T2S_ESHAPE
    assert L.t2s_unet_create(4, 32, 4, 16, 256, 256, ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert L.t2s_unet_param_count(h, ctypes.byref(n)) == 0
    from oracle import unet as U
    assert n.value == U.param_count(8, 32, 4)
    assert L.t2s_unet_workspace_bytes(h, ctypes.byref(n)) == 0 and n.value > 0
    assert L.t2s_unet_bind_workspace(h, None, 0, None) == T.T2S_ENOMEM
    assert L.t2s_unet_destroy(h) == 0


def test_unet_init_params_follow_packing():
    from oracle import unet as U
    L = T.lib()
    h = ctypes.c_void_p()
    assert L.t2s_unet_create(4, 32, 4, 1, 64, 64, ctypes.byref(h)) == 0
    n = U.param_count(8, 32, 4)
    p = np.empty(n, np.float32)
    assert L.t2s_unet_init_params(h, ctypes.c_uint64(7), p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))) == 0
    P = U.unpack(p.astype(np.float64), 8, 32, 4)
    for name, kind, k, ci, co in U.layer_specs(8, 32, 4):
        W, b = P[name]
        assert np.all(b == 0)
        fan_in = k * k * ci if kind == "conv" else ci
        sd = np.sqrt(2.0 / fan_in) * (0.1 if name == "final" else 1.0)
        assert abs(W.std() / sd - 1) < 0.15, name
    q = np.empty(n, np.float32)
    L.t2s_unet_init_params(h, ctypes.c_uint64(7), q.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    assert np.array_equal(p, q)
    L.t2s_unet_destroy(h)


def test_paper_grid_two_map_sets_and_twelve_point_blocks_accepted():
    # 240 x 260 (260 a row length only), two coil-map sets, 12 x 12 blocks (partial at
    # the end of the 260-point axis); the workspace grows with the map sets and holds
    # the intermediate in whole 16-column tiles (272 columns)
    q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((8, 4)))
    phi = q.astype(np.float32)
    masks = (np.random.default_rng(3).random((8, 240, 260)) < 0.05).astype(np.uint8)
    sizes = {}
    for nm in (1, 2):
        code, h = _create(phi, [(240, 260, 7, 1, masks, nm)], block=12)
        assert code == 0, T.t2s_last_error()
        sizes[nm] = T.t2s_plan_workspace_bytes(h)
        T.t2s_plan_destroy(h)
    # one slice: maps C N and seven coefficient vectors K N per map set, 8 bytes each
    assert sizes[2] - sizes[1] >= 8 * 240 * 260 * (7 + 7 * 4)
    code, h = _create(phi, [(240, 260, 7, 1, masks)], block=12)
    tiles = T.t2s_plan_workspace_bytes(h)
    T.t2s_plan_destroy(h)
    assert tiles >= 7 * 4 * 240 * 272 * 8


def test_stream_validation_without_gpu():
    """Streaming entry points check their arguments and the plan state before any HIP call."""
    L = T.lib()
    phi = _phi()
    cls, masks = _classes()
    assert L.t2s_stream_open(None, 0, None, T.T2S_BATCHED) == T.T2S_EINVAL
    assert L.t2s_stream_submit(None, 1, 0, None, None, None, None) == T.T2S_EINVAL
    assert L.t2s_stream_run(None, 0, None, None, None) == T.T2S_EINVAL
    assert L.t2s_stream_close(None) == T.T2S_EINVAL
    code, h = _create(phi, cls)
    assert code == 0
    buf = np.zeros(10, np.complex64)
    # not open: submit / run are state errors
    assert L.t2s_stream_submit(h, 1, 0, buf.ctypes.data, buf.ctypes.data, buf.ctypes.data, None) == T.T2S_ESTATE
    assert L.t2s_stream_run(h, 0, None, None, None) == T.T2S_ESTATE
    # bad class / mode, then the unbound workspace
    assert L.t2s_stream_open(h, 1, None, T.T2S_BATCHED) == T.T2S_EINVAL
    assert L.t2s_stream_open(h, 0, None, T.T2S_PER_SLICE) == T.T2S_EINVAL
    assert L.t2s_stream_open(h, 0, None, T.T2S_BATCHED) == T.T2S_ESTATE
    assert L.t2s_stream_close(h) == 0
    assert L.t2s_plan_destroy(h) == 0
    # two shape classes: streaming needs a one-class plan
    cls2 = cls + [(32, 32, 2, 1, masks[:, :32, :32].copy())]
    code, h = _create(phi, cls2)
    assert code == 0
    assert L.t2s_stream_open(h, 0, None, T.T2S_BATCHED) == T.T2S_EINVAL
    assert L.t2s_plan_destroy(h) == 0


def test_unet_get_shape_without_gpu():
    h = ctypes.c_void_p()
    L = T.lib()
    assert L.t2s_unet_create(5, 16, 3, 4, 32, 48, ctypes.byref(h)) == 0
    K, B, H, W = (ctypes.c_int() for _ in range(4))
    assert L.t2s_unet_get_shape(h, ctypes.byref(K), ctypes.byref(B), ctypes.byref(H), ctypes.byref(W)) == 0
    assert (K.value, B.value, H.value, W.value) == (5, 4, 32, 48)
    assert L.t2s_unet_get_shape(h, None, None, None, None) == 0
    assert L.t2s_unet_get_shape(None, None, None, None, None) == T.T2S_EINVAL
    assert L.t2s_unet_destroy(h) == 0
