"""GPU parity of the particle scheme (kernel sums, velocity, steps, observables)
against the FP64 oracle, through the C ABI.  Needs an MI355X and libvds.so.

Tolerances (float32 GPU vs float64 oracle on the same float32 inputs):
  kernel sums S: max relative 1e-5
  Brownian b = term1 + term2 and velocity v: ||gpu - oracle||_2 / ||oracle||_2 <= 1e-5
    (for v the denominator is max(||v||, ||(1/zeta)(A (x) I) grad Psi||), since
    the total velocity can nearly vanish at steady state); and per particle row
    I, the same ratio over row I alone <= 1e-4, so that one bad row or tile
    cannot hide in the global norm (a row's FP32 group sums and the
    cancellation in x_I S_I - M_I allow up to ~1e-4 on a single row)
  stress: relative Frobenius 1e-4; energy terms: 1e-5 of their magnitude
The same bounds hold for every pair implementation, the FP16-split ones
included (their products keep about 22 significant bits).
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import vds as ovds

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2603_12550_amd as pkg
    return pkg


def _dev(a):
    import torch
    return torch.from_numpy(wl.to_f32(a)).cuda()


def _ctx(pkg, nb, P, h, **kw):
    return pkg.Context(nb, P, h, poison=True, **kw)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


TUNINGS = [(0, 1, 1), (0, 2, 8), (0, 4, 3), (1, 1, 1), (1, 1, 5), (2, 1, 1), (2, 2, 8), (2, 4, 3),
           (3, 1, 1), (3, 2, 8), (3, 4, 3), (4, 1, 1), (4, 2, 8), (4, 1, 3), (4, 2, 5)]
# the default (FP32, 32x32 distance tiles and 4x4 sum blocks), the 16x16 FP32
# form, the FP16-split sums alone and the FP16-split form throughout, at
# benchmark shapes
IMPLS = [None, (0, 4, 16), (2, 4, 16), (3, 2, 8)]


@pytest.mark.parametrize("P", [1, 2, 3, 17, 63, 64, 300])
@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5])
def test_pair_sums_brute_force_small(lib, P, nb):
    q64 = wl.gaussian_bonds(100 + P, nb, P, 0.5)
    q = wl.f32_as_f64(wl.to_f32(q64))
    w64 = wl.random_weights(7 + P, P)
    w = wl.f32_as_f64(wl.to_f32(w64))
    h = 0.45
    x = ovds.particle_major(q)
    S_o, t1_o, t2_o = ovds.brownian_terms(x, w, h)
    b_o = ovds.bond_major(t1_o + t2_o, nb)
    ctx = _ctx(lib, nb, P, h, scheme="explicit")
    for impl, rb, sp in TUNINGS:
        _say(f"pair sums P={P} nb={nb} impl={impl} rb={rb} splits={sp}")
        ctx.set_tuning(impl, rb, sp)
        S, t1, t2 = ctx.pair_sums(_dev(q), _dev(w))
        S, t1, t2 = S.cpu().numpy(), t1.cpu().numpy(), t2.cpu().numpy()
        assert np.max(np.abs(S - S_o) / S_o) < 1e-5
        b = t1.astype(np.float64) + t2
        scale = max(np.linalg.norm(b_o), 1e-3 * math.sqrt(b_o.size) / h ** 2)
        assert np.linalg.norm(b - b_o) / scale < 1e-5, (impl, rb, sp)
        assert np.linalg.norm(t1 - ovds.bond_major(t1_o, nb)) / scale < 1e-5


@pytest.mark.parametrize("nb", [1, 2, 3, 5])
def test_pair_sums_far_particles_mix_folded_and_full_rows(lib, nb):
    """A few particles far from the rest (kappa |x|^2 well above 100 after
    centring) among ordinary ones: the FP32 32x32 kernel takes every distance
    step for the waves holding them and folds the row-norm term out of the
    exponent for the others.  Both kinds of row, and the isolated particles'
    own sums (self term only, up to FP32 underflow), match the oracle for every
    launch shape of that kernel."""
    P, h = 1000, 0.45
    q64 = wl.gaussian_bonds(41 + nb, nb, P, 0.5)
    far = np.array([5, 6, 333, 700, 999])
    rng = np.random.default_rng(9)
    d = rng.normal(size=(nb, far.size, 3))
    q64[:, far, :] += 9.0 * d / np.sqrt((d ** 2).sum(axis=(0, 2)))[None, :, None]  # |offset| = 9 in R^D
    q = wl.f32_as_f64(wl.to_f32(q64))
    w = wl.f32_as_f64(wl.to_f32(wl.random_weights(17, P)))
    x = ovds.particle_major(q)
    kappa = math.log2(math.e) / (2 * h * h)
    xc = x - (w[:, None] * x).sum(axis=0)
    assert (kappa * (xc ** 2).sum(axis=1))[far].min() > 150  # these rows take every step
    S_o, t1_o, t2_o = ovds.brownian_terms(x, w, h)
    b_o = ovds.bond_major(t1_o + t2_o, nb)
    ctx = _ctx(lib, nb, P, h, scheme="explicit")
    for rb, sp in [(1, 1), (2, 4), (1, 3), (2, 8)]:
        _say(f"far particles nb={nb} impl=4 rb={rb} per-CU={sp}")
        ctx.set_tuning(4, rb, sp)
        S, t1, t2 = ctx.pair_sums(_dev(q), _dev(w))
        S, t1, t2 = S.cpu().numpy(), t1.cpu().numpy(), t2.cpu().numpy()
        assert np.max(np.abs(S - S_o) / S_o) < 1e-5
        b = t1.astype(np.float64) + t2
        scale = max(np.linalg.norm(b_o), 1e-3 * math.sqrt(b_o.size) / h ** 2)
        assert np.linalg.norm(b - b_o) / scale < 1e-5, (rb, sp)
        # per particle, against the same global scale: no row may carry the error
        row_err = np.sqrt(((b - b_o) ** 2).sum(axis=(0, 2)))
        assert row_err.max() / scale < 1e-5, (rb, sp, int(row_err.argmax()))


def test_uniform_weights_null_pointer_matches_explicit_uniform(lib):
    P, nb, h = 500, 3, 0.4
    q = wl.to_f32(wl.gaussian_bonds(5, nb, P, 1 / 3))
    ctx = _ctx(lib, nb, P, h)
    S1, a1, b1 = ctx.pair_sums(_dev(q))
    S2, a2, b2 = ctx.pair_sums(_dev(q), _dev(np.full(P, 1.0 / P)))
    assert np.allclose(S1.cpu().numpy(), S2.cpu().numpy(), rtol=1e-6)
    assert np.allclose((a1 + b1).cpu().numpy(), (a2 + b2).cpu().numpy(), rtol=1e-5, atol=1e-5)


def _velocity_check(lib, cfg, rows=None, tuning=None, threads=8):
    P, nb = cfg["P"], cfg["nb"]
    q32 = wl.to_f32(cfg["q0"])
    q = wl.f32_as_f64(q32)
    prob = ovds.problem_from(cfg)
    w = ovds.uniform_weights(P)
    ctx = _ctx(lib, nb, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], potential=cfg["potential"],
               b_max=cfg["b_max"])
    if tuning is not None:
        ctx.set_tuning(*tuning)
    v, diag = ctx.velocity(_dev(q32), diag=True)
    v = v.cpu().numpy().astype(np.float64)
    x = ovds.particle_major(q)
    if rows is None:
        v_o = ovds.velocity(q, w, prob, threads=threads)
        vg, spring = v, ovds.rouse_apply(ovds.rouse_matrix(nb), ovds.grad_potential(q, prob)) / prob.zeta
    else:
        S_all = ovds.density_sums(x, w, prob.h, threads=threads)
        _, t1, t2 = ovds.brownian_terms(x, w, prob.h, rows=rows, S_all=S_all, threads=threads)
        qs = q[:, rows, :]
        g = prob.kT * ovds.bond_major(t1 + t2, nb) + ovds.grad_potential(qs, prob)
        A = ovds.rouse_matrix(nb)
        v_o = ovds.flow_term(qs, prob) - ovds.rouse_apply(A, g) / prob.zeta
        vg = v[:, rows, :]
        spring = ovds.rouse_apply(A, ovds.grad_potential(qs, prob)) / prob.zeta
    denom = max(np.linalg.norm(v_o), np.linalg.norm(spring))
    err = np.linalg.norm(vg - v_o) / denom
    row_num = np.sqrt(((vg - v_o) ** 2).sum(axis=(0, 2)))
    row_den = np.maximum(np.sqrt((v_o ** 2).sum(axis=(0, 2))), np.sqrt((spring ** 2).sum(axis=(0, 2))))
    assert (row_num / row_den).max() < 1e-4, (row_num / row_den).max()
    tau_o = ovds.stress(q, w, prob)
    assert np.linalg.norm(diag["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4
    return err, diag, ctx


@pytest.mark.parametrize("tuning", IMPLS)
def test_velocity_dumbbell_full_size(lib, tuning):
    cfg = wl.dumbbell_shear()  # P = 2000, D = 3, h = 0.3
    _say(f"velocity dumbbell P=2000 tuning {tuning}")
    err, diag, _ = _velocity_check(lib, cfg, tuning=tuning)
    assert err < 1e-5, err


@pytest.mark.parametrize("tuning", IMPLS)
def test_velocity_chain4_full_size_sampled_rows(lib, tuning):
    cfg = wl.chain4_shear()  # P = 20000, D = 9, h = 0.4
    rows = np.random.default_rng(0).choice(cfg["P"], 256, replace=False)
    rows = np.concatenate([rows, [0, cfg["P"] - 1]])
    _say(f"velocity chain4 P=20000 sampled rows tuning {tuning}")
    err, _, _ = _velocity_check(lib, cfg, rows=rows, tuning=tuning)
    assert err < 1e-5, err


def test_fene_state_outside_the_domain_is_rejected(lib):
    # one bond with |q|^2 = 53 >= b_max = 50: every call that evaluates the
    # spring force reports it, and the next valid call works again
    import torch
    cfg = wl.fene_chain6(P=300)
    P = cfg["P"]
    good = wl.to_f32(cfg["q0"])
    bad = good.copy()
    bad[2, 17] = [6.0, 4.0, 1.0]
    kw = dict(G=cfg["G"], dt=cfg["dt"], potential="fene", b_max=cfg["b_max"])
    for scheme in ("explicit", "implicit"):
        ctx = _ctx(lib, 5, P, cfg["h"], scheme=scheme, **kw)
        _say(f"FENE domain check, {scheme}")
        ctx.velocity(_dev(good))
        with pytest.raises(lib.VDSError, match="FENE"):
            ctx.velocity(_dev(bad))
        with pytest.raises(lib.VDSError, match="FENE"):
            ctx.step(_dev(bad))
        with pytest.raises(lib.VDSError, match="FENE"):
            ctx.energy(_dev(bad))
        q = _dev(good)
        ctx.step(q, nsteps=2)
        assert bool(torch.isfinite(q).all().item())


@pytest.mark.parametrize("tuning", IMPLS)
def test_velocity_fene_chain6_sampled_rows(lib, tuning):
    cfg = wl.fene_chain6(P=6000)
    rows = np.random.default_rng(1).choice(cfg["P"], 200, replace=False)
    _say(f"velocity FENE chain6 P=6000 tuning {tuning}")
    err, _, _ = _velocity_check(lib, cfg, rows=rows, tuning=tuning)
    assert err < 1e-5, err


def test_velocity_all_tunings_agree(lib):
    cfg = wl.chain4_shear(P=3000, seed=9)
    for t in TUNINGS:
        _say(f"velocity chain4 P=3000 tuning {t}")
        err, _, _ = _velocity_check(lib, cfg, tuning=t)
        assert err < 1e-5, (t, err)


def test_energy_dissipation_work_match_oracle(lib):
    cfg = wl.chain4_shear(P=1500, seed=3)
    q32 = wl.to_f32(cfg["q0"])
    q = wl.f32_as_f64(q32)
    prob = ovds.problem_from(cfg)
    w = ovds.uniform_weights(cfg["P"])
    ctx = _ctx(lib, 3, cfg["P"], cfg["h"], H=cfg["H"], G=cfg["G"])
    F, Dg, W = ctx.energy(_dev(q32))
    F_o = ovds.free_energy(q, w, prob)
    D_o, W_o = ovds.dissipation_and_work(q, w, prob)
    # F sums terms of magnitude |kT log f| + Psi; compare on that scale
    Sx = ovds.density_sums(ovds.particle_major(q), w, prob.h)
    mag = (w * (np.abs(np.log(Sx)) + ovds.potential(q, prob))).sum()
    assert abs(F - F_o) / mag < 1e-5
    assert abs(Dg - D_o) / D_o < 1e-5
    assert abs(W - W_o) / (abs(W_o) + 1e-3 * D_o) < 1e-4


@pytest.mark.parametrize("tuning", IMPLS)
def test_implicit_steps_match_oracle_trajectory(lib, tuning):
    cfg = wl.chain4_shear(P=3000, seed=12)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    if tuning is not None:
        ctx.set_tuning(*tuning)
    for s in range(5):
        _say(f"implicit step {s} chain4 P=3000 tuning {tuning}")
        d = ctx.step(qg)
        qo, m = ovds.step_implicit(qo, w, prob, threads=8)
        assert 1 <= d["last_iters"] <= 10
        assert _rel(qg.cpu().numpy(), qo) < 1e-5
        tau_o = ovds.stress(qo, w, prob)
        assert np.linalg.norm(d["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4


def test_queued_implicit_steps_match_oracle(lib):
    # several implicit steps in one call run queued on the device (the
    # convergence test in a one-block kernel between iterations, the
    # write-back in a step-end kernel); the trajectory still follows the
    # oracle step by step
    cfg = wl.chain4_shear(P=1500, seed=21)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    _say("queued implicit steps chain4 P=1500, 6 steps in one call")
    d = ctx.step(qg, nsteps=6)
    iters = 0
    for _ in range(6):
        qo, m = ovds.step_implicit(qo, w, prob, threads=8)
        iters += m
    assert d["steps"] == 6
    assert _rel(qg.cpu().numpy(), qo) < 1e-5
    # the device stops at rtol 1e-6, the oracle at 1e-13: the device never
    # takes more iterations
    assert 6 <= d["iters"] <= iters


@pytest.mark.parametrize("predictor", [0, 1])
def test_queued_implicit_steps_across_queues_match_oracle(lib, predictor):
    # 140 steps in one call cross two queue boundaries (64 steps each): the
    # first step of a queue centres with its own mean kernel, the others with
    # the partials the previous step end left; random weights
    cfg = wl.chain4_shear(P=200, seed=23)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w32 = wl.to_f32(wl.random_weights(11, P))
    q32 = wl.to_f32(cfg["q0"])
    qo, wo = wl.f32_as_f64(q32), wl.f32_as_f64(w32)
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit",
               picard_predictor=predictor)
    _say(f"140 queued implicit steps chain4 P=200 predictor {predictor}")
    d = ctx.step(qg, w=_dev(w32), nsteps=140)
    for _ in range(140):
        qo, _ = ovds.step_implicit(qo, wo, prob)
    assert d["steps"] == 140
    assert _rel(qg.cpu().numpy(), qo) < 1e-5


def test_implicit_predictor_same_fixed_point_fewer_iterations(lib):
    # picard_predictor = 1 starts each step after the first of a call from
    # 2 q^n - q^(n-1): the same implicit Euler solution (within the fixed-point
    # tolerance, so within the velocity tolerance of the oracle), reached in
    # fewer iterations
    cfg = wl.chain4_shear(P=1500, seed=23)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    kw = dict(H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    q_plain, q_pred = _dev(q32), _dev(q32)
    _say("implicit predictor chain4 P=1500, 8 steps")
    d_plain = _ctx(lib, 3, P, cfg["h"], **kw).step(q_plain, nsteps=8)
    d_pred = _ctx(lib, 3, P, cfg["h"], picard_predictor=1, **kw).step(q_pred, nsteps=8)
    for _ in range(8):
        qo, _ = ovds.step_implicit(qo, w, prob, threads=8)
    assert _rel(q_pred.cpu().numpy(), qo) < 1e-5
    assert _rel(q_pred.cpu().numpy(), q_plain.cpu().numpy().astype(np.float64)) < 1e-5
    assert d_pred["iters"] < d_plain["iters"]
    assert np.linalg.norm(d_pred["tau"] - d_plain["tau"]) / np.linalg.norm(d_plain["tau"]) < 1e-5


@pytest.mark.parametrize("batch", [1, 2, 3])
def test_queued_implicit_steps_do_not_depend_on_batching(lib, batch):
    # 70 steps (more than one queue of 64): with picard_batch below the
    # iterations a step needs, every step halts the queue and the host
    # finishes it; the iterates are the same kernels on the same inputs, so
    # the trajectory and the iteration counts are identical bit for bit to
    # those of a batch that never halts, and to one step per call
    cfg = wl.chain4_shear(P=700, seed=22)
    P = cfg["P"]
    q32 = wl.to_f32(cfg["q0"])
    kw = dict(H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit", picard_rtol=1e-6)
    ref = _dev(q32)
    ctx_ref = _ctx(lib, 3, P, cfg["h"], picard_batch=12, **kw)
    d_ref = ctx_ref.step(ref, nsteps=70)
    _say(f"queued implicit steps chain4 P=700, 70 steps, picard_batch={batch}")
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], picard_batch=batch, **kw)
    d = ctx.step(qg, nsteps=70)
    assert torch_equal(qg, ref)
    assert (d["steps"], d["iters"], d["last_iters"]) == (d_ref["steps"], d_ref["iters"], d_ref["last_iters"])
    assert d["resid"] == d_ref["resid"]
    q1 = _dev(q32)
    total = 0
    for _ in range(70):
        total += ctx.step(q1)["last_iters"]
    assert torch_equal(q1, ref)
    assert total == d_ref["iters"]


def torch_equal(a, b):
    return bool((a == b).all().item())


@pytest.mark.parametrize("tuning", IMPLS)
def test_implicit_dumbbell_trajectory_and_stress(lib, tuning):
    cfg = wl.dumbbell_shear()
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 1, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    if tuning is not None:
        ctx.set_tuning(*tuning)
    for s in range(6):
        _say(f"implicit step {s} dumbbell P=2000 tuning {tuning}")
        d = ctx.step(qg)
        qo, _ = ovds.step_implicit(qo, w, prob, threads=8)
        assert _rel(qg.cpu().numpy(), qo) < 1e-5
        tau_o = ovds.stress(qo, w, prob)
        assert np.linalg.norm(d["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4


@pytest.mark.parametrize("tuning", IMPLS)
def test_explicit_steps_across_recentring_match_oracle(lib, tuning):
    # 150 explicit steps in one call: the prep kernels centre and pack at
    # steps 0, 64 and 128, the combine kernels pack in between; a strong shear
    # moves the state away from where it was centred
    cfg = wl.chain4_shear(P=400, seed=13)
    prob = ovds.problem_from(cfg)
    prob.G = 5.0 * prob.G
    P = cfg["P"]
    w32 = wl.to_f32(wl.random_weights(9, P))
    q32 = wl.to_f32(cfg["q0"])
    qo, wo = wl.f32_as_f64(q32), wl.f32_as_f64(w32)
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=prob.G, dt=cfg["dt"], scheme="explicit")
    if tuning is not None:
        ctx.set_tuning(*tuning)
    _say(f"150 explicit steps chain4 P=400 tuning {tuning}")
    ctx.step(qg, w=_dev(w32), nsteps=150)
    for _ in range(150):
        qo = ovds.step_explicit(qo, wo, prob)
    assert _rel(qg.cpu().numpy(), qo) < 1e-5


@pytest.mark.parametrize("tuning", IMPLS)
def test_explicit_steps_match_oracle_fene(lib, tuning):
    cfg = wl.fene_chain6(P=700)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 5, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme="explicit", potential="fene",
               b_max=cfg["b_max"])
    if tuning is not None:
        ctx.set_tuning(*tuning)
    _say(f"explicit steps FENE chain6 P=700 tuning {tuning}")
    ctx.step(qg, nsteps=4)
    for _ in range(4):
        qo = ovds.step_explicit(qo, w, prob)
    assert _rel(qg.cpu().numpy(), qo) < 1e-5


@pytest.mark.parametrize("tuning", IMPLS)
def test_queued_implicit_steps_fene_chain6_match_oracle(lib, tuning):
    # D = 15: two FP16 distance slices, written by the prep kernel for a
    # step's first iteration and by the combine kernel for the later ones
    cfg = wl.fene_chain6(P=700)
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 5, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme="implicit", potential="fene",
               b_max=cfg["b_max"], picard_batch=4)
    if tuning is not None:
        ctx.set_tuning(*tuning)
    _say(f"queued implicit steps FENE chain6 P=700 tuning {tuning}")
    d = ctx.step(qg, nsteps=3)
    for _ in range(3):
        qo, _ = ovds.step_implicit(qo, w, prob)
    assert 1 <= d["last_iters"] <= 10
    assert _rel(qg.cpu().numpy(), qo) < 1e-5


@pytest.mark.parametrize("tuning", IMPLS)
def test_implicit_step_full_size_solves_the_implicit_equation(lib, tuning):
    # chain4 at P = 20000: one implicit step on the GPU; on sampled rows the
    # oracle checks (q+ - q*)/dt = u(q+) with q* = q + dt G q (Appendix A)
    cfg = wl.chain4_shear()
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    q0 = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    if tuning is not None:
        ctx.set_tuning(*tuning)
    _say(f"implicit step chain4 P=20000 tuning {tuning}")
    d = ctx.step(qg)
    assert 2 <= d["last_iters"] <= 8
    qp = qg.cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(2).choice(P, 256, replace=False)
    x = ovds.particle_major(qp)
    S_all = ovds.density_sums(x, w, prob.h, threads=8)
    _, t1, t2 = ovds.brownian_terms(x, w, prob.h, rows=rows, S_all=S_all, threads=8)
    g = prob.kT * ovds.bond_major(t1 + t2, 3) + ovds.grad_potential(qp[:, rows], prob)
    u = -ovds.rouse_apply(ovds.rouse_matrix(3), g) / prob.zeta
    qstar = q0[:, rows] + prob.dt * ovds.flow_term(q0[:, rows], prob)
    r = qp[:, rows] - qstar - prob.dt * u
    assert np.linalg.norm(r) / np.linalg.norm(prob.dt * u) < 1e-3
    tau_o = ovds.stress(qp, w, prob)
    assert np.linalg.norm(d["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4


@pytest.mark.parametrize("tuning", IMPLS)
def test_density_at_grid_points(lib, tuning):
    # Appendix A density on the {-2, 0, 2}^D grid (D = 6 here: 729 points)
    nb, P, h = 2, 900, 0.5
    q32 = wl.to_f32(wl.gaussian_bonds(17, nb, P, 1.0))
    q = wl.f32_as_f64(q32)
    grid = np.array(np.meshgrid(*[[-2.0, 0.0, 2.0]] * (3 * nb), indexing="ij")).reshape(3 * nb, -1).T
    f_o = ovds.density_at(grid, q, ovds.uniform_weights(P), h)
    ctx = _ctx(lib, nb, P, h)
    if tuning is not None:
        ctx.set_tuning(*tuning)
    _say(f"density at grid points tuning {tuning}")
    f = ctx.density_at(_dev(q32), _dev(grid)).cpu().numpy()
    assert np.linalg.norm(f - f_o) / np.linalg.norm(f_o) < 1e-5


@pytest.mark.parametrize("tuning", IMPLS)
def test_runs_are_bitwise_deterministic(lib, tuning):
    cfg = wl.chain4_shear(P=4000, seed=4)
    q32 = wl.to_f32(cfg["q0"])
    ctx = _ctx(lib, 3, cfg["P"], cfg["h"], H=cfg["H"], G=cfg["G"])
    if tuning is not None:
        ctx.set_tuning(*tuning)
    a = ctx.velocity(_dev(q32)).cpu().numpy()
    b = ctx.velocity(_dev(q32)).cpu().numpy()
    assert np.array_equal(a, b)


def test_autotune_picks_a_valid_shape(lib):
    cfg = wl.chain4_shear(P=5000, seed=6)
    q32 = wl.to_f32(cfg["q0"])
    ctx = _ctx(lib, 3, cfg["P"], cfg["h"], H=cfg["H"], G=cfg["G"])
    t = ctx.autotune(_dev(q32))
    # the shape only: the default FP32 implementation stays
    assert t["impl"] == 4 and t["rows_per_wave"] in (1, 2) and 1 <= t["col_splits"] <= 32
    err, _, _ = _velocity_check(lib, cfg, tuning=(t["impl"], t["rows_per_wave"], t["col_splits"]))
    assert err < 1e-5


def test_not_converged_status(lib):
    # a cap of one iteration cannot meet the tolerance
    cfg = wl.chain4_shear(P=600, seed=8)
    ctx = _ctx(lib, 3, cfg["P"], cfg["h"], G=cfg["G"], scheme="implicit", picard_max=1, picard_rtol=1e-9)
    with pytest.raises(lib.VDSError) as ei:
        ctx.step(_dev(cfg["q0"]))
    assert ei.value.status == lib._vds.VDS_ERR_NOT_CONVERGED


@pytest.mark.parametrize("P", [2, 3, 17, 300, 1001, 2000])
@pytest.mark.parametrize("nb", [1, 3, 5])
def test_median_bandwidth_matches_oracle(lib, P, nb):
    # eq. model_bandwidth: exact selection over the P^2 ordered pair distances
    # (J = K included); FP32 squared distances against the FP64 oracle
    q32 = wl.to_f32(wl.gaussian_bonds(200 + P, nb, P, 1.0))
    q = wl.f32_as_f64(q32)
    ctx = _ctx(lib, nb, P, 0.4)
    _say(f"median bandwidth P={P} nb={nb}")
    med, h = ctx.median_bandwidth(_dev(q32))
    h_o = ovds.median_bandwidth(q)
    med_o = h_o * math.sqrt(2.0 * math.log(P))
    assert med == pytest.approx(med_o, rel=1e-6, abs=1e-12)
    assert h == pytest.approx(h_o, rel=1e-6, abs=1e-12)


def test_median_bandwidth_rejects_one_particle(lib):
    ctx = _ctx(lib, 1, 1, 0.4)
    with pytest.raises(lib.VDSError) as ei:
        ctx.median_bandwidth(_dev(np.zeros((1, 1, 3))))
    assert ei.value.status == lib._vds.VDS_ERR_ARG


def test_pair_timer_samples_every_stride_th_launch(lib):
    # the bench's roofline comes from these timers: 12 explicit steps are 24
    # pair launches; stride 1 times all of them, stride 5 launches 0, 5, ...,
    # 20; the work counts the P^2 pair-evaluations of each timed launch
    from paper_2603_12550_amd import _vds
    cfg = wl.chain4_shear(P=2000, seed=3)
    P = cfg["P"]
    ctx = _ctx(lib, 3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="explicit")
    q = _dev(cfg["q0"])
    for stride, timed in ((1, 24), (5, 5)):
        ctx.timing_enable(True, stride=stride)
        ctx.step(q, nsteps=12)
        t = ctx.timing_read(_vds.VDS_TIMER_PAIR)
        assert t["launches"] == timed
        assert t["work"] == pytest.approx(timed * float(P) * P)
        assert t["ms"] > 0
    ctx.timing_enable(False)
    ctx.step(q, nsteps=2)
    t = ctx.timing_read(_vds.VDS_TIMER_PAIR)
    assert t["launches"] == 0


@pytest.mark.parametrize("scheme", ["explicit", "implicit"])
def test_step_counts_at_the_boundary(lib, scheme):
    # zero steps change nothing (and evaluate nothing: even a FENE state
    # outside the domain passes), a negative count is rejected, one step
    # matches the oracle
    cfg = wl.fene_chain6(P=200)
    P = cfg["P"]
    prob = ovds.problem_from(cfg)
    ctx = _ctx(lib, 5, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme=scheme, potential="fene",
               b_max=cfg["b_max"])
    bad = wl.to_f32(cfg["q0"]).copy()
    bad[1, 3] = [7.0, 1.0, 1.0]
    qb = _dev(bad)
    ctx.step(qb, nsteps=0)
    assert np.array_equal(qb.cpu().numpy(), bad)
    with pytest.raises(lib.VDSError):
        ctx.step(qb, nsteps=-1)
    q32 = wl.to_f32(cfg["q0"])
    qg = _dev(q32)
    ctx.step(qg, nsteps=1)
    qo = wl.f32_as_f64(q32)
    qo = ovds.step_explicit(qo, ovds.uniform_weights(P), prob) if scheme == "explicit" else \
        ovds.step_implicit(qo, ovds.uniform_weights(P), prob)[0]
    assert _rel(qg.cpu().numpy(), qo) < 1e-5
