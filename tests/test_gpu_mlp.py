"""GPU parity of the learned reduced step (include/vds_mlp.h): forward, loss and
gradients against the FP64 oracle's hand-written backward pass, Adam against
the oracle's update, BF16 inference against FP32, and the checked rollout with
its fallback to the particle scheme.

Tolerances: loss relative 1e-5; gradients relative Frobenius 1e-4 per tensor
(FP32 MFMA products); Adam parameters after three steps relative 1e-5 (at the
learned step's shape, on the elements whose update is determined); BF16
inference within 1e-3 of the oracle's BF16 forward and within 3e-2 of FP32
(8-bit mantissas); rollout stress within 1e-2 of the plain scheme."""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mlp as omlp

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


def _flat(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def _unflat(v, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = v[o:o + a * b].reshape(b, a)
        o += a * b
        bb = v[o:o + b]
        o += b
        out.append((W, bb))
    return out


def _case(nin=37, w=32, nout=29, n=50, seed=3):
    sizes = [nin, w, w, nout]
    layers = wl.mlp_init(seed, sizes)
    rng = np.random.default_rng(seed)
    layers = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in layers]
    layers = [(wl.f32_as_f64(wl.to_f32(W)), wl.f32_as_f64(wl.to_f32(b))) for W, b in layers]
    X = wl.f32_as_f64(wl.to_f32(rng.standard_normal((n, nin))))
    T = wl.f32_as_f64(wl.to_f32(rng.standard_normal((n, nout))))
    return sizes, layers, X, T


def _dev(a):
    import torch
    return torch.from_numpy(wl.to_f32(a)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_loss_and_gradients_match_oracle(lib):
    sizes, layers, X, T = _case()
    m = lib.Mlp(sizes[0], sizes[1], sizes[3], 64)
    m.set_params(_dev(_flat(layers)))
    Y = m.forward(_dev(X)).cpu().numpy()
    Y_o, _ = omlp.forward(layers, X)
    assert _rel(Y, Y_o) < 1e-5
    loss = m.loss_grad(_dev(X), _dev(T))
    loss_o, grads_o = omlp.backward(layers, X, T)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    g = _unflat(m.get_grads().cpu().numpy().astype(np.float64), sizes)
    for (gW, gb), (oW, ob) in zip(g, grads_o):
        assert _rel(gW, oW) < 1e-4
        assert _rel(gb, ob) < 1e-4


def test_gradients_and_adam_at_the_learned_step_shape(lib):
    # the learned step's own shape: 541 inputs (3 x 180 POD coefficients and
    # the log shear rate), width 128, 540 outputs; batch 64
    sizes, layers, X, T = _case(nin=541, w=128, nout=540, n=64, seed=11)
    m = lib.Mlp(541, 128, 540, 64)
    m.set_params(_dev(_flat(layers)))
    _say("MLP 541-128-128-540, batch 64: loss and gradients")
    Y = m.forward(_dev(X)).cpu().numpy()
    assert _rel(Y, omlp.forward(layers, X)[0]) < 1e-5
    loss = m.loss_grad(_dev(X), _dev(T))
    loss_o, grads_o = omlp.backward(layers, X, T)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    g = _unflat(m.get_grads().cpu().numpy().astype(np.float64), sizes)
    for (gW, gb), (oW, ob) in zip(g, grads_o):
        assert _rel(gW, oW) < 1e-4
        assert _rel(gb, ob) < 1e-4
    # three Adam steps.  Adam's first steps move each parameter by about lr
    # times the sign of its gradient, so an element whose gradient lies within
    # the FP32 rounding of zero has no determined update: the comparison takes
    # the elements whose oracle gradient exceeds 1e-3 of its tensor's RMS in
    # every step (all but a small fraction)
    _say("MLP 541-128-128-540: three Adam steps")
    mo, vo = omlp.adam_init(layers)
    lo = layers
    keep = np.ones(_flat(layers).size, dtype=bool)
    for t in range(1, 4):
        m.loss_grad(_dev(X), _dev(T))
        m.adam_step(1e-3)
        _, go = omlp.backward(lo, X, T)
        keep &= np.concatenate([np.concatenate([np.abs(gW).reshape(-1) > 1e-3 * np.sqrt((gW ** 2).mean()),
                                                np.abs(gb) > 1e-3 * np.sqrt((gb ** 2).mean())])
                                for gW, gb in go])
        lo, mo, vo = omlp.adam_step(lo, go, mo, vo, t, lr=1e-3)
    assert keep.mean() > 0.99
    got = m.get_params().cpu().numpy().astype(np.float64)
    want = _flat(lo)
    assert np.linalg.norm((got - want)[keep]) / np.linalg.norm(want[keep]) < 1e-5


def test_bf16_inference_matches_the_oracle_bf16_forward(lib):
    # the BF16 inference arithmetic (weights and layer inputs rounded to bfloat16,
    # FP32 sums) against the oracle's forward with the same roundings done in
    # NumPy.  The GPU sums in FP32 and may round a hidden activation that lies
    # within its FP32 error of a bfloat16 tie the other way: about one element
    # in 10^3, each moving the output by ~2^-9 of one term, hence 1e-3
    sizes, layers, X, _ = _case(nin=541, w=128, nout=540, n=16, seed=4)
    m = lib.Mlp(541, 128, 540, 16)
    m.set_params(_dev(_flat(layers)))
    y16 = m.forward(_dev(X), bf16=True).cpu().numpy()
    assert _rel(y16, omlp.forward_bf16(layers, X)) < 1e-3


def test_bf16_inference_tracks_fp32(lib):
    sizes, layers, X, _ = _case(nin=541, w=128, nout=540, n=16, seed=4)
    m = lib.Mlp(541, 128, 540, 16)
    m.set_params(_dev(_flat(layers)))
    y32 = m.forward(_dev(X)).cpu().numpy()
    y16 = m.forward(_dev(X), bf16=True).cpu().numpy()
    assert _rel(y16, y32) < 3e-2
    y1 = m.forward(_dev(X[:1]), bf16=True).cpu().numpy()   # batch of one, as in the rollout
    assert _rel(y1, y16[:1]) < 1e-6


@pytest.mark.parametrize("shape", [(541, 128, 540), (601, 64, 600), (4001, 32, 4000)])
def test_fused_learned_steps_match_layer_by_layer(lib, shape):
    # vds_mlp_predict_steps against the BF16 layer kernels (vds_mlp_forward)
    # with the scaling and update done in torch: same roundings, FP32 sums in
    # another order.  The shapes take the three paths: weights resident on
    # chip (nin <= 544, width <= 128, nout <= 576), one workgroup streaming
    # the weights from L2, and layer by layer.
    import torch
    nin, w, nout = shape
    sizes, layers, _, _ = _case(nin=nin, w=w, nout=nout, n=1, seed=6)
    layers = [(W * 0.5, b) for W, b in layers]
    m = lib.Mlp(nin, w, nout, 16)
    m.set_params(_dev(_flat(layers)))
    rng = np.random.default_rng(7)
    xs, xsc = _dev(rng.standard_normal(nin) * 0.1), _dev(0.5 + rng.random(nin))
    ys, ysc = _dev(rng.standard_normal(nout) * 1e-3), _dev(1e-3 * (0.5 + rng.random(nout)))
    m.set_scaling(xs, xsc, ys, ysc)
    p0 = _dev(rng.standard_normal(nout))
    log_rate = -0.3
    ref = p0.clone()
    for _ in range(5):
        x = (torch.cat([ref, torch.tensor([log_rate], dtype=torch.float32, device=ref.device)]) - xs) / xsc
        y = m.forward(x[None].contiguous(), bf16=True)[0]
        ref = ref + (y * ysc + ys)
    got = m.predict_steps(p0.clone(), log_rate, 5)
    inc_ref = (ref - p0).cpu().numpy().astype(np.float64)
    inc = (got - p0).cpu().numpy().astype(np.float64)
    assert _rel(inc, inc_ref) < 1e-3
    one = m.predict_steps(p0.clone(), log_rate, 0)
    assert bool((one == p0).all().item())


def test_adam_steps_match_oracle(lib):
    sizes, layers, X, T = _case(seed=5)
    m = lib.Mlp(sizes[0], sizes[1], sizes[3], 64)
    m.set_params(_dev(_flat(layers)))
    mo, vo = omlp.adam_init(layers)
    lo = layers
    for t in range(1, 4):
        m.loss_grad(_dev(X), _dev(T))
        m.adam_step(1e-2)
        _, g = omlp.backward(lo, X, T)
        lo, mo, vo = omlp.adam_step(lo, g, mo, vo, t, lr=1e-2)
    got = m.get_params().cpu().numpy().astype(np.float64)
    assert _rel(got, _flat(lo)) < 1e-5


def test_training_epochs_reduce_loss(lib):
    import torch
    rng = np.random.default_rng(6)
    X = rng.standard_normal((512, 9))
    T = np.tanh(X @ rng.standard_normal((9, 8)))
    m = lib.Mlp(9, 32, 8, 64)
    m.set_params(_dev(_flat(wl.mlp_init(7, [9, 32, 32, 8]))))
    from paper_2603_12550_amd import learned
    losses = learned.train(m, _dev(X), _dev(T), epochs=60, batch=64, lr=3e-3, seed=1)
    assert losses[-1] < 0.2 * losses[0]


def test_input_noise_is_seeded_and_off_by_default(lib):
    # vds_mlp_set_input_noise: sigma = 0 is the plain epoch (bit for bit), the
    # same seed gives the same epoch, another seed another one; with the
    # learning rate 0 the epoch's loss grows with the noise
    rng = np.random.default_rng(8)
    nout = 12
    X = rng.standard_normal((256, nout + 1))
    T = 0.1 * rng.standard_normal((256, nout))
    init = _dev(_flat(wl.mlp_init(3, [nout + 1, 16, 16, nout])))

    def epoch(sigma, seed, lr=3e-3, set_noise=True):
        m = lib.Mlp(nout + 1, 16, nout, 64)
        m.set_params(init)
        m.fit_scaling(_dev(X), _dev(T))
        if set_noise:
            m.set_input_noise(sigma, seed)
        loss = m.train_epoch(_dev(X), _dev(T), 64, lr)
        return loss, m.get_params().cpu().numpy()

    l_plain, p_plain = epoch(0.0, 0, set_noise=False)
    l0, p0 = epoch(0.0, 5)
    assert l0 == l_plain and np.array_equal(p0, p_plain)
    la, pa = epoch(2.0, 7)
    lb, pb = epoch(2.0, 7)
    lc, pc = epoch(2.0, 8)
    assert la == lb and np.array_equal(pa, pb)
    assert not np.array_equal(pa, pc)
    assert epoch(2.0, 7, lr=0.0)[0] > epoch(0.0, 7, lr=0.0)[0]
    m = lib.Mlp(nout + 1, 16, nout, 64)
    with pytest.raises(lib.VDSError):
        m.set_input_noise(-1.0)
    m2 = lib.Mlp(nout + 2, 16, nout, 64)
    with pytest.raises(lib.VDSError):
        m2.set_input_noise(1.0)


def _pipeline(lib, P=400, R=20, rates=(0.5, 1.0, 2.0), nsteps=300, width=64, epochs=150):
    import torch
    from paper_2603_12550_amd import learned
    cfgs = []
    states = []
    for i, r in enumerate(rates):
        ctx = lib.Context(3, P, 0.4, G=wl.shear_gradient(r), dt=1e-3, scheme="explicit")
        q0 = torch.from_numpy(wl.to_f32(wl.gaussian_bonds(60, 3, P, 1 / 3))).cuda()
        cfgs.append((ctx, q0, r))
        states += learned.run_states(ctx, q0, nsteps, 10)
    U, eig = cfgs[0][0].pod_basis(learned.snapshot_matrix(states), R)
    trajs = [(learned.reduced_trajectory(ctx, U, q0, nsteps), math.log(r)) for ctx, q0, r in cfgs]
    m = lib.Mlp(3 * R + 1, width, 3 * R, 256)
    m.set_params(_dev(_flat(wl.mlp_init(8, [3 * R + 1, width, width, 3 * R]))))
    X, T = learned.training_set(m, trajs)
    losses = learned.train(m, X, T, epochs=epochs, batch=64, lr=2e-3, seed=2)
    return cfgs, U, m, trajs, losses


def test_learned_rollout_tracks_plain_scheme_and_falls_back(lib):
    import torch
    _say("learned-step pipeline P=400 R=20")
    cfgs, U, m, trajs, losses = _pipeline(lib)
    assert losses[-1] < 0.1 * losses[0]
    ctx, q0, r = cfgs[1]
    # plain scheme reference at t_end
    q = q0.clone()
    ctx.step(q, nsteps=300)
    tau_ref = ctx.stress(q)
    p = ctx.pod_project(U, q0)
    st = m.rollout(ctx, U, p, math.log(r), nsteps=300, check_every=50, resid_tol=0.5, energy_tol=0.5)
    _say("rollout", st)
    assert st["checks"] == 6
    assert np.linalg.norm(st["tau"] - tau_ref) / np.linalg.norm(tau_ref) < 1e-2
    # a tolerance of zero rejects every window: the rollout is the plain scheme, re-projected
    p = ctx.pod_project(U, q0)
    st0 = m.rollout(ctx, U, p, math.log(r), nsteps=300, check_every=50, resid_tol=0.0, energy_tol=0.5)
    assert st0["fallbacks"] == st0["checks"] == 6
    assert np.linalg.norm(st0["tau"] - tau_ref) / np.linalg.norm(tau_ref) < 1e-2
    # a broken network (scaling replaced, increments ten times larger) fails the residual check
    R = U.shape[0]
    xs = torch.zeros(3 * R + 1, device="cuda")
    m.set_scaling(xs, torch.ones_like(xs), torch.zeros(3 * R, device="cuda"),
                  10.0 * torch.ones(3 * R, device="cuda"))
    p = ctx.pod_project(U, q0)
    st10 = m.rollout(ctx, U, p, math.log(r), nsteps=100, check_every=50, resid_tol=0.5, energy_tol=0.5)
    assert st10["fallbacks"] == st10["checks"] == 2


def test_learned_rollout_fene_chain6(lib):
    # the same pipeline on the 6-bead FENE chain (five bonds: its own basis and
    # network); the POD-Galerkin model has no FENE form, the rollout checks
    # itself against the plain scheme
    import torch
    from paper_2603_12550_amd import learned
    P, R, nsteps = 400, 20, 300
    cfg = wl.fene_chain6(P=P)

    def mk(r):
        return lib.Context(5, P, cfg["h"], G=wl.shear_gradient(r), dt=cfg["dt"], scheme="explicit",
                           potential="fene", b_max=cfg["b_max"])

    _say("learned-step pipeline, FENE chain6 P=400 R=20")
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    rates = (0.5, 1.0, 2.0)
    states = []
    for r in rates:
        states += learned.run_states(mk(r), q0, nsteps, 10)
    U, _ = mk(1.0).pod_basis(learned.snapshot_matrix(states), R)
    trajs = [(learned.reduced_trajectory(mk(r), U, q0, nsteps), math.log(r)) for r in rates]
    m = lib.Mlp(5 * R + 1, 64, 5 * R, 256)
    m.set_params(_dev(_flat(wl.mlp_init(8, [5 * R + 1, 64, 64, 5 * R]))))
    X, T = learned.training_set(m, trajs)
    losses = learned.train(m, X, T, epochs=150, batch=64, lr=2e-3, seed=2)
    assert losses[-1] < 0.1 * losses[0]
    ctx = mk(1.0)
    q = q0.clone()
    ctx.step(q, nsteps=nsteps)
    tau_ref = ctx.stress(q)
    st = m.rollout(ctx, U, ctx.pod_project(U, q0), 0.0, nsteps=nsteps, check_every=50, resid_tol=0.5,
                   energy_tol=0.5)
    _say("rollout", st)
    assert st["checks"] == 6
    assert np.linalg.norm(st["tau"] - tau_ref) / np.linalg.norm(tau_ref) < 1e-2
    st0 = m.rollout(ctx, U, ctx.pod_project(U, q0), 0.0, nsteps=nsteps, check_every=50, resid_tol=0.0,
                    energy_tol=0.5)
    assert st0["fallbacks"] == st0["checks"] == 6
    assert np.linalg.norm(st0["tau"] - tau_ref) / np.linalg.norm(tau_ref) < 1e-2


def test_learned_step_gains_over_the_reduced_model_without_it(lib):
    # the method without the network is the POD-Galerkin model, whose operators
    # are rebuilt every window by a kernel GEMM of O(P^2 R) products; the
    # learned rollout evaluates pairs only at its checks.  Same windows (50
    # steps), same basis: both stay within 1e-2 of the plain scheme, and the
    # learned one does a fraction of the O(P^2) work (at the bench's size,
    # P = 20000 and R = 180, it is 15x faster than the plain scheme against
    # 2.7x for the Galerkin model)
    from paper_2603_12550_amd import _vds
    cfgs, U, m, trajs, losses = _pipeline(lib)
    ctx, q0, r = cfgs[1]
    q = q0.clone()
    ctx.step(q, nsteps=300)
    tau_ref = ctx.stress(q)

    def measured(run):
        ctx.timing_enable(True)
        tau = run()
        pair = ctx.timing_read(_vds.VDS_TIMER_PAIR)
        kg = ctx.timing_read(_vds.VDS_TIMER_KGEMM)
        ctx.timing_enable(False)
        err = np.linalg.norm(tau - tau_ref) / np.linalg.norm(tau_ref)
        return err, pair, kg

    err_l, pair_l, kg_l = measured(lambda: m.rollout(ctx, U, ctx.pod_project(U, q0), math.log(r), nsteps=300,
                                                     check_every=50, resid_tol=0.5, energy_tol=0.5)["tau"])
    err_g, pair_g, kg_g = measured(lambda: lib.Rom(ctx, U).run(ctx.pod_project(U, q0), 300, 50))
    _say("learned", err_l, pair_l, kg_l, "galerkin", err_g, pair_g, kg_g)
    assert err_l < 1e-2 and err_g < 1e-2
    assert kg_l["launches"] == 0 and kg_g["launches"] == 6
    assert pair_l["launches"] == 2 * 7  # the velocity at the start and after each of 6 windows
    flop_per_pair = 4 * 9 + 4
    work_l = pair_l["work"] * flop_per_pair
    work_g = pair_g["work"] * flop_per_pair + kg_g["work"]
    assert work_l < 0.5 * work_g
