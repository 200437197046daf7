"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: single operator applications are FP32 FFT chains, checked at 1e-5
relative L2; whole ADMM runs at the 1e-4 relative L2 the build targets on the
subspace coefficients.
"""

import sys

import numpy as np
import pytest

import paper_1809_04195_amd as T
from oracle import t2s as O
from gpu_helpers import crandn, random_problem, rel

pytestmark = pytest.mark.gpu


def _plan(phi, classes, **kw):
    return T.Plan(phi, classes, **kw)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu(gpu):
    return gpu


OPS_SHAPES = [
    (64, 64, 4, 16, 3),
    (32, 16, 2, 6, 2),
    (48, 96, 3, 10, 4),
    (192, 320, 6, 20, 5),
    (256, 256, 8, 80, 4),
]


@pytest.mark.parametrize("ny,nz,C,Tn,K", OPS_SHAPES)
def test_normal_operator_and_adjoint(ny, nz, C, Tn, K):
    import torch
    _say(f"normal/adjoint parity ny={ny} nz={nz} C={C} T={Tn} K={K}")
    S = 2
    phi, sens, masks, ksp = random_problem(ny * 7 + nz, ny, nz, C, Tn, K, S=S)
    plan = _plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=S, masks=masks)], lam=0.01, rho=0.1)
    plan.load(0, 0, sens, ksp)
    rng = np.random.default_rng(5)
    a = crandn(rng, S, K, ny, nz)
    a_d = torch.from_numpy(a).cuda()
    out = torch.empty_like(a_d)
    T.t2s_apply_normal(plan.handle, 0, 0, S, a_d, out, 0.1)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    b0 = plan.read(0, 0, S, T.T2S_ADJOINT)
    m = masks.astype(bool)
    psi = O.space_time_kernel(phi, m)
    for s in range(S):
        ref = O.normal_psi(a[s], sens[s], psi) + 0.1 * a[s].astype(np.complex128)
        e = rel(got[s], ref)
        assert e < 1e-5, f"normal op slice {s}: {e}"
        refb = O.adjoint(ksp[s], sens[s], phi, m)
        eb = rel(b0[s], refb)
        assert eb < 1e-5, f"adjoint slice {s}: {eb}"
    plan.close()


# every supported FFT length as row length (nz) and as column length (ny), C = 1-2
LENGTH_SHAPES = [(16, 512), (512, 16), (32, 384), (384, 32), (48, 320), (320, 48), (96, 160), (160, 96),
                 (128, 192), (192, 128), (256, 64), (64, 256)]


@pytest.mark.parametrize("ny,nz", LENGTH_SHAPES)
def test_normal_operator_every_length(ny, nz):
    import torch
    K, C, Tn = 2, 2 if ny * nz <= 16384 else 1, 6
    _say(f"normal-operator parity ny={ny} nz={nz} C={C} K={K}")
    phi, sens, masks, ksp = random_problem(ny + 3 * nz, ny, nz, C, Tn, K, S=1, frac=0.3)
    plan = _plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=1, masks=masks)], lam=0.01, rho=0.1, block=16)
    plan.load(0, 0, sens, ksp)
    a = crandn(np.random.default_rng(ny * nz), 1, K, ny, nz)
    a_d = torch.from_numpy(a).cuda()
    out = torch.empty_like(a_d)
    T.t2s_apply_normal(plan.handle, 0, 0, 1, a_d, out, 0.0)
    torch.cuda.synchronize()
    psi = O.space_time_kernel(phi, masks.astype(bool))
    e = rel(out.cpu().numpy()[0], O.normal_psi(a[0], sens[0], psi))
    _say(f"  rel L2 {e:.3e}")
    assert e < 1e-5
    plan.close()


@pytest.mark.parametrize("K", [6, 7, 8])
def test_normal_operator_and_llr_large_k(K):
    import torch
    _say(f"normal operator and LLR prox at K={K} (64x64, C=2)")
    phi, sens, masks, ksp = random_problem(40 + K, 64, 64, 2, 12, K, S=1, frac=0.3)
    plan = _plan(phi, [dict(ny=64, nz=64, ncoils=2, nslices=1, masks=masks)], lam=0.01, rho=0.1)
    plan.load(0, 0, sens, ksp)
    rng = np.random.default_rng(K)
    a = crandn(rng, 1, K, 64, 64)
    a_d = torch.from_numpy(a).cuda()
    out = torch.empty_like(a_d)
    T.t2s_apply_normal(plan.handle, 0, 0, 1, a_d, out, 0.1)
    torch.cuda.synchronize()
    psi = O.space_time_kernel(phi, masks.astype(bool))
    ref = O.normal_psi(a[0], sens[0], psi) + 0.1 * a[0].astype(np.complex128)
    assert rel(out.cpu().numpy()[0], ref) < 1e-5
    base = crandn(rng, 1, 2, 64, 64)
    v = (np.einsum("sjyz,sjk->skyz", base, crandn(rng, 1, 2, K)) + 0.3 * crandn(rng, 1, K, 64, 64)).astype(np.complex64)
    vd = torch.from_numpy(v).cuda()
    T.t2s_apply_llr(plan.handle, 0, 0, 1, vd, out, 0.9, [(5, 2)])
    torch.cuda.synchronize()
    e = rel(out.cpu().numpy()[0], O.llr_prox(v[0], 0.9, (5, 2), 8))
    _say(f"  LLR rel L2 {e:.3e}")
    assert e < 1e-5
    plan.close()


@pytest.mark.parametrize("K,b", [(1, 8), (2, 4), (3, 8), (4, 8), (5, 8), (4, 16), (3, 4)])
def test_llr_prox(K, b):
    import torch
    _say(f"llr prox parity K={K} b={b}")
    ny, nz = 64, 128 if b != 16 else 64
    phi, sens, masks, ksp = random_problem(3, ny, nz, 1, max(K, 2), K, S=2)
    plan = _plan(phi, [dict(ny=ny, nz=nz, ncoils=1, nslices=2, masks=masks)], lam=0.01, rho=0.1, block=b)
    rng = np.random.default_rng(K * 10 + b)
    # low-rank-ish blocks plus noise so thresholds hit the spectrum in the middle
    base = crandn(rng, 2, 1, ny, nz) * crandn(rng, 2, K, 1, 1)
    v = (base + 0.3 * crandn(rng, 2, K, ny, nz)).astype(np.complex64)
    tau = 0.9 * b / 8
    shifts = [(3 % b, 5 % b), (b - 1, 0)]
    vd = torch.from_numpy(v).cuda()
    out = torch.empty_like(vd)
    T.t2s_apply_llr(plan.handle, 0, 0, 2, vd, out, tau, shifts)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for s in range(2):
        ref = O.llr_prox(v[s], tau, shifts[s], b)
        e = rel(got[s], ref)
        assert e < 1e-5, (s, e)
    # tau = 0 is the identity
    T.t2s_apply_llr(plan.handle, 0, 0, 2, vd, out, 0.0, shifts)
    torch.cuda.synchronize()
    assert rel(out.cpu().numpy(), v) < 1e-6
    plan.close()


def _slice64():
    from synth import make_config
    d = make_config("slice64_c4_t16_k3")
    return d["cfg"], d["phi"], d["classes"][0]


def test_admm_slice64_parity():
    _say("ADMM parity: 64x64 C4 T16 K3, 20 outer x 5 CG, seed 0")
    cfg, phi, cl = _slice64()
    plan = _plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)],
                 lam=cfg["lam"], rho=cfg["rho"], block=cfg["block"], n_outer=cfg["n_outer"], n_cg=cfg["n_cg"],
                 seed=cfg["seed"])
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.reconstruct()
    alpha = plan.read(0, 0, 1)[0]
    z = plan.read(0, 0, 1, T.T2S_Z)[0]
    ref = O.admm(cl.ksp[0], cl.sens[0], phi, cl.masks.astype(bool), cfg["lam"], cfg["rho"], cfg["block"],
                 cfg["n_outer"], cfg["n_cg"], cfg["seed"], g=0)
    e = rel(alpha, ref.alpha)
    ez = rel(z, ref.z)
    _say(f"  rel L2 alpha {e:.3e}  z {ez:.3e}")
    assert e < 1e-4 and ez < 1e-4
    rep = plan.report(0, 0)
    h = ref.history[-1]
    assert rep["outer_iterations"] == cfg["n_outer"]
    assert abs(rep["r_primal"] - h["r_primal"]) <= 1e-3 * h["r_primal"] + 1e-7
    assert abs(rep["r_dual"] - h["r_dual"]) <= 1e-3 * h["r_dual"] + 1e-7
    plan.close()


@pytest.mark.parametrize("ny,nz,C,Tn,K", [(96, 32, 2, 6, 3), (320, 16, 2, 6, 4), (384, 32, 3, 8, 5)])
def test_admm_ragged_column_workgroups(ny, nz, C, Tn, K):
    """Column lengths whose pass-B workgroups do not fill whole waves (12 x 20 threads
    for 320 and 384, 21 x 12 for 96): the CG step length is reduced over them."""
    _say(f"ADMM parity ny={ny} nz={nz} C={C} T={Tn} K={K}, 4 outer x 3 CG, 2 slices")
    phi, sens, masks, ksp = random_problem(ny + nz + K, ny, nz, C, Tn, K, S=2, frac=0.3)
    plan = _plan(phi, [dict(ny=ny, nz=nz, ncoils=C, nslices=2, masks=masks)], lam=0.02, rho=0.1, n_outer=4,
                 n_cg=3, seed=5)
    plan.load(0, 0, sens, ksp)
    plan.reconstruct()
    got = plan.read(0, 0, 2)
    plan.close()
    for s in range(2):
        ref = O.admm(ksp[s], sens[s], phi, masks.astype(bool), 0.02, 0.1, 8, 4, 3, 5, g=s)
        e = rel(got[s], ref.alpha)
        _say(f"  slice {s}: rel L2 {e:.3e}")
        assert e < 1e-4, (s, e)


def test_batched_equals_per_slice_bitwise():
    _say("batched vs per-slice launches, 3 slices 64x64")
    phi, sens, masks, ksp = random_problem(11, 64, 64, 3, 8, 3, S=3, frac=0.3)
    outs = []
    for mode in (T.T2S_BATCHED, T.T2S_PER_SLICE):
        plan = _plan(phi, [dict(ny=64, nz=64, ncoils=3, nslices=3, masks=masks)], lam=0.05, rho=0.1,
                     n_outer=4, n_cg=3, seed=9)
        plan.load(0, 0, sens, ksp)
        plan.reconstruct(mode)
        outs.append(plan.read(0, 0, 3))
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_multiclass_parity():
    _say("two shape classes in one plan (64x64 C4, 32x48 C2), 2 slices each")
    phiA, sA, mA, kA = random_problem(21, 64, 64, 4, 8, 3, S=2, frac=0.25)
    _, sB, mB, kB = random_problem(22, 32, 48, 2, 8, 3, S=2, frac=0.25)
    # same basis for both classes (plan-wide)
    kB = kB  # samples are plain inputs
    plan = _plan(phiA, [dict(ny=64, nz=64, ncoils=4, nslices=2, masks=mA),
                        dict(ny=32, nz=48, ncoils=2, nslices=2, masks=mB)],
                 lam=0.02, rho=0.1, n_outer=6, n_cg=4, seed=3)
    plan.load(0, 0, sA, kA)
    plan.load(1, 0, sB, kB)
    plan.reconstruct()
    for ci, (sens, masks, ksp) in enumerate([(sA, mA, kA), (sB, mB, kB)]):
        got = plan.read(ci, 0, 2)
        for s in range(2):
            g = ci * 2 + s
            ref = O.admm(ksp[s], sens[s], phiA, masks.astype(bool), 0.02, 0.1, 8, 6, 4, 3, g=g)
            e = rel(got[s], ref.alpha)
            assert e < 1e-4, (ci, s, e)
    plan.close()


def test_warm_start_parity():
    _say("warm start (set_initial) parity, 64x64 C4 K3")
    cfg, phi, cl = _slice64()
    rng = np.random.default_rng(2)
    m = cl.masks.astype(bool)
    b0 = O.adjoint(cl.ksp[0], cl.sens[0], phi, m)
    a0 = (1.5 * b0 + 0.01 * crandn(rng, *b0.shape)).astype(np.complex64)
    plan = _plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)],
                 lam=cfg["lam"], rho=cfg["rho"], n_outer=8, n_cg=5, seed=cfg["seed"])
    plan.load(0, 0, cl.sens, cl.ksp)
    plan.set_initial(0, 0, a0[None])
    plan.reconstruct()
    got = plan.read(0, 0, 1)[0]
    ref = O.admm(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["rho"], 8, 8, 5, cfg["seed"], g=0, alpha0=a0)
    e = rel(got, ref.alpha)
    assert e < 1e-4, e
    plan.close()


def test_tolerance_mode_replay_parity():
    _say("tolerance mode: GPU decisions replayed by the oracle, 64x64 C4 K3")
    cfg, phi, cl = _slice64()
    m = cl.masks.astype(bool)
    plan = _plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)],
                 lam=cfg["lam"], rho=cfg["rho"], n_outer=300, n_cg=5, seed=cfg["seed"], tol=1e-4,
                 freeze_window=5, freeze_stall=0.05, check_every=5)
    plan.load(0, 0, cl.sens, cl.ksp)
    code = plan.reconstruct()
    rep = plan.report(0, 0)
    _say(f"  GPU: code {code} outer {rep['outer_iterations']} k_freeze {rep['k_freeze']} "
         f"r_p {rep['r_primal']:.3e} r_d {rep['r_dual']:.3e}")
    got = plan.read(0, 0, 1)[0]
    ref = O.admm(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["rho"], 8, 300, 5, cfg["seed"], g=0,
                 replay=(rep["k_freeze"], rep["outer_iterations"]))
    e = rel(got, ref.alpha)
    _say(f"  replay rel L2 {e:.3e}")
    assert e < 1e-4
    if code == T.T2S_OK:
        assert rep["converged"] == 1 and max(rep["r_primal"], rep["r_dual"]) <= 1e-4
    own = O.admm(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["rho"], 8, 300, 5, cfg["seed"], g=0, tol=1e-4,
                 check_every=5)
    _say(f"  oracle's own decisions: k_freeze {own.k_freeze} outer {own.n_outer}")
    plan.close()
    # the GPU's stop rule takes the oracle's decisions (within one decision interval)
    assert abs(own.k_freeze - rep["k_freeze"]) <= 5 and abs(own.n_outer - rep["outer_iterations"]) <= 5, (own, rep)


def test_tolerance_mode_on_a_side_stream_with_device_inputs():
    import torch
    _say("tolerance mode on a non-blocking torch stream, device inputs, vs the default stream")
    cfg, phi, cl = _slice64()
    kw = dict(lam=cfg["lam"], rho=cfg["rho"], n_outer=300, n_cg=5, seed=cfg["seed"], tol=1e-4, freeze_window=5,
              freeze_stall=0.05, check_every=5)
    classes = [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=1, masks=cl.masks)]
    ref_plan = _plan(phi, classes, **kw)
    ref_plan.load(0, 0, cl.sens, cl.ksp)
    ref_plan.reconstruct(T.T2S_BATCHED_GRAPH)
    ref, ref_rep = ref_plan.read(0, 0, 1), ref_plan.report(0, 0)
    ref_plan.close()
    plan = _plan(phi, classes, **kw)
    side = torch.cuda.Stream()
    ds, dk = torch.from_numpy(cl.sens).cuda(), torch.from_numpy(cl.ksp).cuda()
    side.wait_stream(torch.cuda.current_stream())
    T.t2s_load_slices(plan.handle, 0, 0, 1, ds, dk, side)
    T.t2s_reconstruct(plan.handle, T.T2S_BATCHED_GRAPH, side)
    side.synchronize()
    got, rep = plan.read(0, 0, 1, stream=side), plan.report(0, 0)
    plan.close()
    _say(f"  side stream: outer {rep['outer_iterations']} freeze {rep['k_freeze']}; default: "
         f"{ref_rep['outer_iterations']} {ref_rep['k_freeze']}")
    assert (rep["outer_iterations"], rep["k_freeze"]) == (ref_rep["outer_iterations"], ref_rep["k_freeze"])
    assert np.array_equal(got, ref)


def test_tolerance_mode_empty_slice_stops_first_check():
    _say("tolerance mode: a slice with no signal next to a normal one")
    cfg, phi, cl = _slice64()
    m = cl.masks.astype(bool)
    sens = np.concatenate([cl.sens, cl.sens])
    ksp = np.concatenate([cl.ksp, np.zeros_like(cl.ksp)])
    plan = _plan(phi, [dict(ny=cl.ny, nz=cl.nz, ncoils=cl.ncoils, nslices=2, masks=cl.masks)],
                 lam=cfg["lam"], rho=cfg["rho"], n_outer=300, n_cg=5, seed=cfg["seed"], tol=1e-4,
                 freeze_window=5, freeze_stall=0.05, check_every=5)
    plan.load(0, 0, sens, ksp)
    plan.reconstruct()
    r0, r1 = plan.report(0, 0), plan.report(0, 1)
    _say(f"  normal slice: outer {r0['outer_iterations']} freeze {r0['k_freeze']}; empty slice: {r1}")
    assert r1["outer_iterations"] == 5 and r1["converged"] == 1 and r1["r_primal"] == 0.0
    got = plan.read(0, 0, 2)
    assert not got[1].any()
    ref = O.admm(cl.ksp[0], cl.sens[0], phi, m, cfg["lam"], cfg["rho"], 8, 300, 5, cfg["seed"], g=0,
                 replay=(r0["k_freeze"], r0["outer_iterations"]))
    assert rel(got[0], ref.alpha) < 1e-4
    plan.close()


def test_nonfinite_host_input_rejected():
    phi, sens, masks, ksp = random_problem(4, 32, 32, 2, 4, 2, S=1)
    plan = _plan(phi, [dict(ny=32, nz=32, ncoils=2, nslices=1, masks=masks)], lam=0.01, rho=0.1)
    bad = ksp.copy()
    bad[0, 0, 3] = np.nan
    with pytest.raises(T.T2SError) as ei:
        plan.load(0, 0, sens, bad)
    assert ei.value.code == T.T2S_ENONFINITE
    plan.close()


def _run_sched(phi, sens, masks, ksp, mode, sched=None, reps=1, between=None):
    S = sens.shape[0]
    plan = _plan(phi, [dict(ny=64, nz=64, ncoils=sens.shape[1], nslices=S, masks=masks)], lam=0.05, rho=0.1,
                 n_outer=4, n_cg=3, seed=17)
    if sched is not None:
        T.t2s_set_schedule(plan.handle, 0, *sched)
    outs = []
    for r in range(reps):
        plan.load(0, 0, sens, ksp)
        plan.reconstruct(mode)
        outs.append(plan.read(0, 0, S))
        if between is not None:
            between(plan)
    plan.close()
    return outs


def test_chunked_schedules_bitwise():
    _say("chunked pass launches over 1-3 streams vs one launch per pass")
    phi, sens, masks, ksp = random_problem(31, 64, 64, 3, 8, 3, S=5, frac=0.3)
    ref = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED)[0]
    for sched in [(2, 1), (2, 2), (1, 3), (3, 2), (4, 4)]:
        got = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED, sched)[0]
        assert np.array_equal(got, ref), sched


def test_workgroup_orders_bitwise():
    _say("XCD-grouped workgroup orders of passes A and C vs the plain order")
    phi, sens, masks, ksp = random_problem(34, 64, 64, 3, 8, 3, S=8, frac=0.3)
    outs = []
    for order in range(4):
        plan = _plan(phi, [dict(ny=64, nz=64, ncoils=3, nslices=8, masks=masks)], lam=0.05, rho=0.1, n_outer=4,
                     n_cg=3, seed=17)
        T.t2s_set_order(plan.handle, 0, order)
        assert T.t2s_get_order(plan.handle, 0) == order
        plan.load(0, 0, sens, ksp)
        plan.reconstruct(T.T2S_BATCHED_GRAPH if order % 2 else T.T2S_BATCHED)
        outs.append(plan.read(0, 0, 8))
        plan.close()
    for order in range(1, 4):
        assert np.array_equal(outs[order], outs[0]), order


def test_every_kernel_schedule_flag_combination_bitwise():
    _say("all 16 kernel schedule flag combinations (XCD orders of passes A/C/B, pass C's LDS buffers) at 32 x 256")
    phi, sens, masks, ksp = random_problem(36, 32, 256, 3, 8, 3, S=4, frac=0.3)
    outs = []
    for order in range(16):
        plan = _plan(phi, [dict(ny=32, nz=256, ncoils=3, nslices=4, masks=masks)], lam=0.05, rho=0.1, n_outer=3,
                     n_cg=3, seed=18)
        T.t2s_set_order(plan.handle, 0, order)
        plan.load(0, 0, sens, ksp)
        plan.reconstruct(T.T2S_BATCHED_GRAPH if order % 2 else T.T2S_BATCHED)
        outs.append(plan.read(0, 0, 4))
        plan.close()
    assert np.abs(outs[0]).max() > 0
    for order in range(1, 16):
        assert np.array_equal(outs[order], outs[0]), order


def test_slice_offset_splits_volume_bitwise():
    _say("a 4-slice plan vs two 2-slice plans with global slice offsets 0 and 2")
    phi, sens, masks, ksp = random_problem(35, 64, 64, 3, 8, 3, S=4, frac=0.3)
    whole = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED)[0]
    parts = []
    for first in (0, 2):
        plan = _plan(phi, [dict(ny=64, nz=64, ncoils=3, nslices=2, masks=masks)], lam=0.05, rho=0.1, n_outer=4,
                     n_cg=3, seed=17)
        T.t2s_set_slice_offset(plan.handle, 0, first)
        plan.load(0, 0, sens[first:first + 2], ksp[first:first + 2])
        plan.reconstruct(T.T2S_PER_SLICE)
        parts.append(plan.read(0, 0, 2))
        plan.close()
    assert np.array_equal(np.concatenate(parts), whole)


def test_graph_replay_matches_eager():
    import torch
    _say("hipGraph replay of the outer iteration vs eager launches, 3 replays with eager work between")
    phi, sens, masks, ksp = random_problem(32, 64, 64, 3, 8, 3, S=4, frac=0.3)
    ref = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED)[0]

    def eager_work(plan):
        a = torch.ones((1, 3, 64, 64), dtype=torch.complex64, device="cuda")
        o = torch.empty_like(a)
        T.t2s_apply_normal(plan.handle, 0, 0, 1, a, o, 0.0)
        torch.cuda.synchronize()

    for sched in [None, (2, 2)]:
        outs = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED_GRAPH, sched, reps=3, between=eager_work)
        for i, got in enumerate(outs):
            assert np.array_equal(got, ref), (sched, i)


def test_autotune_schedule_valid_and_exact():
    _say("autotuner picks a schedule; results unchanged")
    phi, sens, masks, ksp = random_problem(33, 64, 64, 3, 8, 3, S=6, frac=0.3)
    ref = _run_sched(phi, sens, masks, ksp, T.T2S_BATCHED)[0]
    plan = _plan(phi, [dict(ny=64, nz=64, ncoils=3, nslices=6, masks=masks)], lam=0.05, rho=0.1, n_outer=4, n_cg=3,
                 seed=17)
    plan.load(0, 0, sens, ksp)
    T.t2s_autotune(plan.handle, 2)
    ch, ns = T.t2s_get_schedule(plan.handle, 0)
    _say(f"  picked chunk={ch} streams={ns}")
    assert 0 <= ch <= 6 and 1 <= ns <= 4
    plan.reconstruct(T.T2S_BATCHED_GRAPH)
    assert np.array_equal(plan.read(0, 0, 6), ref)
    plan.close()
