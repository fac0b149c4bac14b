"""Pins of the oracle's POD, reduced model and learned-step pieces against what
the mathematics fixes: known SVD factors, special cases where the reduced model
is exact, the paper's literal index sums, finite differences.  CPU only."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import mlp, pod, rom, vds


def test_pod_recovers_known_factors():
    # X = Q diag(sigma) W^T with known orthonormal Q, W: the basis spans Q[:, :R]
    # and lambda_i = sigma_i^2 (best rank-R approximation, Section 1.3)
    rng = np.random.default_rng(0)
    n, m, R = 300, 40, 7
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sig = np.sort(rng.uniform(0.1, 10, m))[::-1]
    X = Q @ np.diag(sig) @ W.T
    U, lam = pod.pod_basis(X, R)
    assert np.allclose(lam, sig ** 2, rtol=1e-12)
    assert pod.subspace_distance(U, Q[:, :R]) < 1e-10
    assert np.allclose(U.T @ U, np.eye(R), atol=1e-13)
    # discarded energy: ||X - U U^T X||_F^2 = sum_{i > R} sigma_i^2
    E = X - U @ (U.T @ X)
    assert (E * E).sum() == pytest.approx((sig[R:] ** 2).sum(), rel=1e-10)
    assert pod.remaining_energy(lam)[R - 1] == pytest.approx((sig[R:] ** 2).sum() / (sig ** 2).sum(), rel=1e-10)


def test_subspace_distance_is_the_sine_of_the_largest_principal_angle():
    # Planes in R^6 at known principal angles: span(e1, e2) against
    # span(cos a e1 + sin a e3, cos b e2 + sin b e4) has principal angles a and b,
    # so the distance is sin(max(a, b)); a rotation of the whole space, a change
    # of basis inside either plane or swapping the arguments leaves it unchanged.
    rng = np.random.default_rng(17)
    e = np.eye(6)
    for a, b in ((0.3, 0.0), (0.1, 0.7), (1.2, 0.4), (math.pi / 2, 0.2)):
        U1 = e[:, :2]
        U2 = np.stack([math.cos(a) * e[:, 0] + math.sin(a) * e[:, 2],
                       math.cos(b) * e[:, 1] + math.sin(b) * e[:, 3]], axis=1)
        want = math.sin(max(a, b))
        assert pod.subspace_distance(U1, U2) == pytest.approx(want, abs=1e-14)
        assert pod.subspace_distance(U2, U1) == pytest.approx(want, abs=1e-14)
        Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
        B1, _ = np.linalg.qr(rng.standard_normal((2, 2)))
        B2, _ = np.linalg.qr(rng.standard_normal((2, 2)))
        assert pod.subspace_distance(Q @ U1 @ B1, Q @ U2 @ B2) == pytest.approx(want, abs=1e-13)
    # one shared direction and one orthogonal one: the largest angle is pi/2
    assert pod.subspace_distance(e[:, [0, 1]], e[:, [0, 4]]) == pytest.approx(1.0, abs=1e-15)


def test_snapshot_matrix_column_order_and_round_trip():
    q0 = wl.gaussian_bonds(1, 3, 10, 1.0)
    q1 = wl.gaussian_bonds(2, 3, 10, 1.0)
    X = pod.snapshot_matrix([q0, q1])
    assert X.shape == (30, 6)
    assert np.array_equal(X[:, 4], q1[1].reshape(-1))      # column (l=1, k=1)
    assert X[3 * 4 + 2, 0] == q0[0, 4, 2]                  # row (I=4, alpha=2)
    U, _ = pod.pod_basis(np.random.default_rng(3).standard_normal((30, 30)), 30)
    assert np.allclose(pod.reconstruct(U, pod.project(U, q0), 10), q0, atol=1e-13)


def _small_case(P=12, nb=2, seed=5):
    q = wl.gaussian_bonds(seed, nb, P, 0.5)
    prob = vds.Problem(nb=nb, h=0.6, dt=1e-3, G=wl.shear_gradient(1.0), H=np.array([1.0, 2.0][:nb]))
    return q, prob


def test_row_blocked_operators_equal_the_literal_and_factored_sums():
    # the row-blocked evaluation (used at sizes where the kernel matrix does not
    # fit in memory) against the paper's literal index sums and the factored
    # form, with ragged blocks and threads
    q, prob = _small_case(P=13)
    P = q.shape[1]
    rng = np.random.default_rng(8)
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, 9)))
    _, B1_l, B2_l = rom.operators_literal(U, q, prob)
    for block, threads in ((5, 1), (4, 3), (13, 1), (64, 2)):
        B1, B2 = rom.brownian_rows(U, q, vds.uniform_weights(P), prob.h, block=block, threads=threads)
        assert np.allclose(B1, B1_l, rtol=1e-11, atol=1e-12), block
        assert np.allclose(B2, B2_l, rtol=1e-11, atol=1e-12), block
    w = wl.random_weights(3, P)
    F1, F2 = rom.brownian(U, q, w, prob.h)
    B1, B2 = rom.brownian_rows(U, q, w, prob.h, block=6, threads=2)
    assert np.allclose(B1, F1, rtol=1e-12, atol=1e-13) and np.allclose(B2, F2, rtol=1e-12, atol=1e-13)


def test_factored_operators_equal_the_papers_literal_sums():
    q, prob = _small_case()
    P = q.shape[1]
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, 8)))
    XH_l, B1_l, B2_l = rom.operators_literal(U, q, prob)
    XH = rom.hydro(U, prob.G, P)
    B1, B2 = rom.brownian(U, q, vds.uniform_weights(P), prob.h)
    assert np.allclose(XH, XH_l, atol=1e-13)
    assert np.allclose(B1, B1_l, rtol=1e-11, atol=1e-12)
    assert np.allclose(B2, B2_l, rtol=1e-11, atol=1e-12)


def test_hydro_operator_closed_forms():
    rng = np.random.default_rng(7)
    P = 20
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, 6)))
    # G = identity gives U^T U = I; shear gives sum_I U_(I1)s U_(I2)t
    assert np.allclose(rom.hydro(U, np.eye(3), P), np.eye(6), atol=1e-13)
    XH = rom.hydro(U, wl.shear_gradient(1.0), P)
    assert np.allclose(XH, U[0::3].T @ U[1::3], atol=1e-14)


def test_full_rank_rom_reproduces_full_explicit_vds():
    # R = P d, any orthogonal U, freeze every step: the reduced model is the full
    # explicit scheme written in another basis (Section 2.4 approximations are exact)
    q, prob = _small_case(P=10)
    P = q.shape[1]
    w = vds.uniform_weights(P)
    U, _ = np.linalg.qr(np.random.default_rng(8).standard_normal((3 * P, 3 * P)))
    steps = 5
    qf, _ = vds.run(q, w, prob, steps, scheme="explicit")
    p = rom.rom_run(U, q, w, prob, steps, freeze_every=1)
    assert np.allclose(pod.reconstruct(U, p, P), qf, rtol=1e-11, atol=1e-13)


def test_rom_exact_without_noise_or_flow_in_invariant_subspace():
    # kT = 0 and G = 0: each step is p+ = p - (dt/zeta) A diag(H) p across bonds,
    # so a state inside span U stays there and the reduced run is exact for any U
    P = 15
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, 5)))
    p0 = rng.standard_normal((2, 5))
    q0 = pod.reconstruct(U, p0, P)
    prob = vds.Problem(nb=2, h=0.5, dt=1e-2, kT=0.0, H=np.array([1.0, 3.0]))
    steps = 40
    p = rom.rom_run(U, q0, vds.uniform_weights(P), prob, steps, freeze_every=7)
    M = np.eye(2) - (prob.dt / prob.zeta) * vds.rouse_matrix(2) @ np.diag(prob.H)
    expect = np.linalg.matrix_power(M, steps) @ p0
    assert np.allclose(p, expect, rtol=1e-12, atol=1e-13)


def test_exact_windows_match_the_closed_form_without_noise_or_flow():
    # kT = 0, G = 0: dp/dt = -(1/zeta) A diag(H) p across bonds, so
    # p(t) = V exp(t Lambda) V^-1 p(0) with the eigenpairs of -(1/zeta) A diag(H),
    # whatever the window lengths
    P = 15
    rng = np.random.default_rng(19)
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, 5)))
    p0 = rng.standard_normal((3, 5))
    q0 = pod.reconstruct(U, p0, P)
    prob = vds.Problem(nb=3, h=0.5, dt=1e-2, kT=0.0, H=np.array([1.0, 2.0, 3.0]))
    lam, V = np.linalg.eig(-vds.rouse_matrix(3) @ np.diag(prob.H) / prob.zeta)
    t = 0.9
    expect = np.real(V @ np.diag(np.exp(t * lam)) @ np.linalg.inv(V)) @ p0
    for windows in ([0.9], [0.3, 0.3, 0.3], [0.1, 0.5, 0.25, 0.05]):
        p = rom.rom_run_windows(U, q0, vds.uniform_weights(P), prob, windows)
        assert np.allclose(p, expect, rtol=1e-12, atol=1e-13), windows


def test_exact_windows_and_euler_agree_to_first_order():
    # the same freeze schedule: explicit Euler inside the windows differs from the
    # exact solution by O(dt), so halving dt halves the difference
    q, prob = _small_case(P=14)
    P = q.shape[1]
    U, _ = np.linalg.qr(np.random.default_rng(20).standard_normal((3 * P, 8)))
    w = vds.uniform_weights(P)
    exact = rom.rom_run_windows(U, q, w, prob, [0.02, 0.02, 0.02])
    diffs = []
    for dt in (2e-3, 1e-3):
        pr = vds.Problem(nb=prob.nb, h=prob.h, dt=dt, G=prob.G, kT=prob.kT, H=prob.H)
        n = int(round(0.02 / dt))
        p = rom.rom_run(U, q, w, pr, 3 * n, freeze_every=n)
        diffs.append(np.linalg.norm(p - exact) / np.linalg.norm(exact))
    assert 0.4 < diffs[1] / diffs[0] < 0.6, diffs
    assert diffs[0] < 0.05


def test_weighted_brownian_operator_reduces_to_uniform():
    q, prob = _small_case(P=14)
    P = q.shape[1]
    U, _ = np.linalg.qr(np.random.default_rng(10).standard_normal((3 * P, 6)))
    a = rom.brownian(U, q, vds.uniform_weights(P), prob.h)
    b = rom.brownian(U, q, np.full(P, 3.0), prob.h)
    assert np.allclose(a[0], b[0], rtol=1e-12) and np.allclose(a[1], b[1], rtol=1e-12)


def _mlp_case():
    layers = wl.mlp_init(3, [7, 16, 16, 5])
    rng = np.random.default_rng(4)
    layers = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in layers]
    X = rng.standard_normal((11, 7))
    Y = rng.standard_normal((11, 5))
    return layers, X, Y


def test_silu_values():
    assert mlp.silu(np.array(0.0)) == 0.0
    assert mlp.silu_grad(np.array(0.0)) == pytest.approx(0.5)
    z = 1.3
    assert mlp.silu(np.array(z)) == pytest.approx(z / (1 + math.exp(-z)))


def test_mlp_gradients_match_central_differences():
    layers, X, Y = _mlp_case()
    _, grads = mlp.backward(layers, X, Y)
    eps = 1e-6
    rng = np.random.default_rng(5)
    for li, (W, b) in enumerate(layers):
        for _ in range(6):
            i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
            Lp = [(w.copy(), c.copy()) for w, c in layers]; Lp[li][0][i, j] += eps
            Lm = [(w.copy(), c.copy()) for w, c in layers]; Lm[li][0][i, j] -= eps
            fd = (mlp.loss(Lp, X, Y) - mlp.loss(Lm, X, Y)) / (2 * eps)
            assert fd == pytest.approx(grads[li][0][i, j], rel=1e-6, abs=1e-10)
        i = rng.integers(b.shape[0])
        Lp = [(w.copy(), c.copy()) for w, c in layers]; Lp[li][1][i] += eps
        Lm = [(w.copy(), c.copy()) for w, c in layers]; Lm[li][1][i] -= eps
        fd = (mlp.loss(Lp, X, Y) - mlp.loss(Lm, X, Y)) / (2 * eps)
        assert fd == pytest.approx(grads[li][1][i], rel=1e-6, abs=1e-10)


def test_adam_first_step_moves_each_parameter_by_lr():
    # bias-corrected first step: m_hat = g, v_hat = g^2, step = lr * g / (|g| + eps)
    layers, X, Y = _mlp_case()
    _, grads = mlp.backward(layers, X, Y)
    m, v = mlp.adam_init(layers)
    new, _, _ = mlp.adam_step(layers, grads, m, v, 1, lr=1e-3, eps=0.0)
    for (W, _), (W1, _), (gW, _) in zip(layers, new, grads):
        assert np.allclose(W - W1, 1e-3 * np.sign(gW), rtol=1e-12)


def test_training_reduces_loss():
    layers, X, Y = _mlp_case()
    m, v = mlp.adam_init(layers)
    L0 = mlp.loss(layers, X, Y)
    for t in range(1, 201):
        _, g = mlp.backward(layers, X, Y)
        layers, m, v = mlp.adam_step(layers, g, m, v, t, lr=3e-3)
    assert mlp.loss(layers, X, Y) < 0.2 * L0


def test_midpoint_freeze_is_second_order_in_the_window():
    # differences between runs with windows M and M/2 (the time step fixed):
    # they halve with M for operators frozen at the window's start (first
    # order) and quarter for operators at the predicted midpoint, whether the
    # midpoint state is predicted by reduced steps or extrapolated from the
    # last two window starts (second order; a wrong extrapolation coefficient
    # or sign leaves the prediction first order, and the ratio near 2)
    q, prob = _small_case(P=14)
    P = q.shape[1]
    U, _ = np.linalg.qr(np.random.default_rng(21).standard_normal((3 * P, 10)))
    w = vds.uniform_weights(P)
    steps = 128
    runs = {(mid, M): rom.rom_run(U, q, w, prob, steps, freeze_every=M, midpoint=mid)
            for mid in (False, True, "extrapolated") for M in (8, 16, 32, 64)}
    scale = np.linalg.norm(runs[(False, 8)])
    for mid, lo, hi in ((False, 1.8, 2.3), (True, 3.6, 4.6), ("extrapolated", 3.3, 4.6)):
        d = [np.linalg.norm(runs[(mid, M)] - runs[(mid, M // 2)]) / scale for M in (16, 32, 64)]
        assert lo < d[1] / d[0] < hi and lo < d[2] / d[1] < hi, (mid, d)
    # a window of one step has no midpoint to predict: the schedules agree
    a = rom.rom_run(U, q, w, prob, 10, freeze_every=1)
    for mid in (True, "extrapolated"):
        assert np.array_equal(a, rom.rom_run(U, q, w, prob, 10, freeze_every=1, midpoint=mid))
    # within the first window there is no earlier start to extrapolate from:
    # both midpoint forms predict by reduced steps
    a = rom.rom_run(U, q, w, prob, 12, freeze_every=16, midpoint=True)
    assert np.array_equal(a, rom.rom_run(U, q, w, prob, 12, freeze_every=16, midpoint="extrapolated"))


def test_bf16_rounding_matches_torch_bfloat16():
    # round to nearest even at 8 significant bits, checked against torch's CPU
    # conversion on ordinary values, exact ties, both tie directions, signs and
    # tiny/large magnitudes
    import torch
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 1.0 + 2.0 ** -9,
                         0.0, -0.0, 65504.0, 3.0e38]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and goes to the even 1
    assert mlp.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def test_bf16_forward_reduces_to_the_fp64_forward_on_bf16_exact_operands():
    # weights and inputs already representable in bfloat16, and hidden
    # activations rounded by the bf16 form only: with a single linear layer
    # the two forwards agree exactly
    rng = np.random.default_rng(13)
    W = mlp.bf16_round(rng.standard_normal((7, 11)))
    b = rng.standard_normal(7).astype(np.float32).astype(np.float64)
    X = mlp.bf16_round(rng.standard_normal((5, 11)))
    y, _ = mlp.forward([(W, b)], X)
    assert np.array_equal(mlp.forward_bf16([(W, b)], X), y)
    # two layers: the hidden activation is rounded, so they differ by about 2^-9
    W2 = mlp.bf16_round(rng.standard_normal((3, 7)))
    y2, _ = mlp.forward([(W, b), (W2, b[:3])], X)
    y2b = mlp.forward_bf16([(W, b), (W2, b[:3])], X)
    assert 0 < np.abs(y2b - y2).max() < 2.0 ** -6 * np.abs(y2).max()
