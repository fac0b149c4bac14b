"""Pins of the FP64 oracle's particle scheme against facts the paper and the
mathematics fix (closed forms, exact identities, the paper's printed values).
CPU only."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import vds

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _brute_phi(x, w, h):
    """Phi_w by plain Python loops (independent of the oracle's vectorised sums)."""
    P = x.shape[0]
    tot = 0.0
    for K in range(P):
        s = 0.0
        for J in range(P):
            r2 = sum((x[K, a] - x[J, a]) ** 2 for a in range(x.shape[1]))
            s += w[J] * math.exp(-r2 / (2 * h * h))
        tot += w[K] * math.log(s)
    return tot


def test_rouse_matrix_matches_definition_and_spectrum():
    A = vds.rouse_matrix(3)
    assert np.array_equal(A, np.array([[2., -1, 0], [-1, 2, -1], [0, -1, 2]]))
    ev = np.sort(np.linalg.eigvalsh(A))
    assert np.allclose(ev, [2 - math.sqrt(2), 2, 2 + math.sqrt(2)], atol=1e-14)
    assert vds.rouse_matrix(1)[0, 0] == 2.0


def test_single_particle_has_no_brownian_drift():
    x = np.array([[0.3, -1.2, 0.7]])
    S, t1, t2 = vds.brownian_terms(x, np.ones(1), 0.4)
    assert S[0] == pytest.approx(1.0)
    assert np.abs(t1).max() == 0.0 and np.abs(t2).max() == 0.0


def test_two_particles_closed_form():
    # b_1 = -(2/h^2) Delta e / (1 + e), e = exp(-|Delta|^2 / 2h^2), uniform weights
    rng = np.random.default_rng(0)
    for D in (3, 9):
        x = rng.standard_normal((2, D)) * 0.5
        h = 0.37
        _, t1, t2 = vds.brownian_terms(x, np.full(2, 0.5), h)
        delta = x[0] - x[1]
        e = math.exp(-(delta @ delta) / (2 * h * h))
        expect = -(2 / h ** 2) * delta * e / (1 + e)
        assert np.allclose((t1 + t2)[0], expect, rtol=1e-13, atol=1e-15)
        assert np.allclose((t1 + t2)[1], -expect, rtol=1e-13, atol=1e-15)


def test_translation_invariance_sum_rule():
    # Phi_w is translation invariant, so sum_I w_I b_I = 0
    rng = np.random.default_rng(1)
    x = rng.standard_normal((60, 9)) * 0.6
    w = wl.random_weights(2, 60)
    _, t1, t2 = vds.brownian_terms(x, w, 0.4)
    tot = (w[:, None] * (t1 + t2)).sum(0)
    assert np.abs(tot).max() < 1e-13 * np.abs(t1).max()


def test_virial_identity():
    # sum_I w_I x_I (x) b_I = -(1/h^2) sum_K (w_K/S_K) sum_J w_J K_KJ Delta_KJ (x) Delta_KJ
    rng = np.random.default_rng(3)
    P, D, h = 40, 6, 0.5
    x = rng.standard_normal((P, D)) * 0.7
    w = wl.random_weights(4, P)
    S, t1, t2 = vds.brownian_terms(x, w, h)
    lhs = np.einsum("i,ia,ib->ab", w, x, t1 + t2)
    rhs = np.zeros((D, D))
    for K in range(P):
        sK = 0.0
        acc = np.zeros((D, D))
        for J in range(P):
            dlt = x[K] - x[J]
            kk = math.exp(-(dlt @ dlt) / (2 * h * h))
            sK += w[J] * kk
            acc += w[J] * kk * np.outer(dlt, dlt)
        rhs += (w[K] / sK) * acc
    rhs *= -1.0 / h ** 2
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-14)


def test_brownian_term_is_scaled_gradient_of_blob_energy():
    # b_I = (1/w_I) dPhi_w/dx_I, Phi_w = sum_K w_K log sum_J w_J K(x_K - x_J)
    rng = np.random.default_rng(5)
    P, D, h = 9, 3, 0.45
    x = rng.standard_normal((P, D)) * 0.5
    w = wl.random_weights(6, P)
    _, t1, t2 = vds.brownian_terms(x, w, h)
    b = t1 + t2
    # the oracle's own Phi_w against the plain double loop
    assert vds.blob_energy(x, w, h) == pytest.approx(_brute_phi(x, w, h), rel=1e-13, abs=1e-15)
    eps = 1e-5
    for I in (0, 4, 8):
        for a in range(D):
            xp = x.copy(); xp[I, a] += eps
            xm = x.copy(); xm[I, a] -= eps
            fd = (_brute_phi(xp, w, h) - _brute_phi(xm, w, h)) / (2 * eps) / w[I]
            assert fd == pytest.approx(b[I, a], rel=1e-7, abs=1e-9)


def test_permutation_and_rotation_equivariance():
    rng = np.random.default_rng(7)
    P, D, h = 50, 9, 0.4
    x = rng.standard_normal((P, D)) * 0.6
    w = wl.random_weights(8, P)
    _, t1, t2 = vds.brownian_terms(x, w, h)
    perm = rng.permutation(P)
    _, u1, u2 = vds.brownian_terms(x[perm], w[perm], h)
    assert np.allclose(u1 + u2, (t1 + t2)[perm], rtol=1e-12, atol=1e-13)
    Q, _ = np.linalg.qr(rng.standard_normal((D, D)))
    _, r1, r2 = vds.brownian_terms(x @ Q, w, h)
    assert np.allclose(r1 + r2, (t1 + t2) @ Q, rtol=1e-11, atol=1e-12)


def test_weight_scale_invariance_and_uniform_reduction():
    # the bracket of eq. model_DymRepPar uses counts, not weights: w = c/P gives the same b
    rng = np.random.default_rng(9)
    x = rng.standard_normal((30, 6))
    _, a1, a2 = vds.brownian_terms(x, np.full(30, 1 / 30), 0.5)
    _, c1, c2 = vds.brownian_terms(x, np.full(30, 7.0), 0.5)
    assert np.allclose(a1 + a2, c1 + c2, rtol=1e-13)
    # and the literal uniform form: sum grad K / sum K for both terms
    K = np.exp(-((x[:, None] - x[None]) ** 2).sum(-1) / (2 * 0.25))
    gradK = -(x[:, None] - x[None]) / 0.25 * K[..., None]
    lit1 = gradK.sum(1) / K.sum(1)[:, None]
    lit2 = (gradK / K.sum(0)[None, :, None]).sum(1)
    assert np.allclose(a1, lit1, rtol=1e-12) and np.allclose(a2, lit2, rtol=1e-12)


def test_equilibrium_stress_of_initial_condition():
    # q ~ N(0, k_B T / H_k) gives tau = n (N-1) k_B T Id up to sampling error
    P = 200000
    H = np.array([1.0, 2.0, 3.0])
    q = wl.gaussian_bonds(11, 3, P, 1.0 / H)
    prob = vds.Problem(nb=3, h=0.4, H=H)
    tau = vds.stress(q, vds.uniform_weights(P), prob)
    assert np.allclose(tau, 3.0 * np.eye(3), atol=0.03)


def test_fene_force_is_gradient_of_fene_potential():
    prob = vds.Problem(nb=2, h=0.4, H=np.array([1.0, 1.5]), potential="fene", b_max=10.0)
    q = wl.gaussian_bonds(12, 2, 5, 1.0)
    gp = vds.grad_potential(q, prob)
    eps = 1e-6
    for k in range(2):
        for I in range(5):
            for a in range(3):
                qp = q.copy(); qp[k, I, a] += eps
                qm = q.copy(); qm[k, I, a] -= eps
                fd = (vds.potential(qp, prob)[I] - vds.potential(qm, prob)[I]) / (2 * eps)
                assert fd == pytest.approx(gp[k, I, a], rel=1e-7, abs=1e-9)


def test_hookean_dumbbell_tracks_exact_moment_ode_under_shear():
    # Exact second-moment ODE of the Fokker-Planck equation (Hookean, linear drift):
    # dC/dt = G C + C G^T - (4H/zeta) C + (4 kT/zeta) I for a dumbbell (A = 2).
    # Started from the particles' empirical C(0) it must track VDS over t <= 0.1
    # up to the kernel regularisation bias (~1%); the shear increment of tau_12 is
    # the sign/convention check of G.
    import scipy.linalg
    P = 600
    cfg = wl.dumbbell_shear(P=P, seed=21)
    prob = vds.problem_from(cfg)
    prob.h, prob.dt = 0.5, 2e-3
    w = vds.uniform_weights(P)
    q0 = cfg["q0"]
    qT, _ = vds.run(q0.copy(), w, prob, 50, scheme="explicit", threads=4)
    tau0 = vds.stress(q0, w, prob)
    tauT = vds.stress(qT, w, prob)
    G = prob.G
    L = (np.kron(G, np.eye(3)) + np.kron(np.eye(3), G)) - (4 / prob.zeta) * np.eye(9)
    c = (4 / prob.zeta) * np.eye(3).reshape(-1)
    C0 = tau0.reshape(-1)
    # closed form of the affine ODE: C(t) = e^{Lt} C0 + L^{-1}(e^{Lt} - I) c
    E = scipy.linalg.expm(L * 0.1)
    CT = (E @ C0 + np.linalg.solve(L, (E - np.eye(9)) @ c)).reshape(3, 3)
    assert np.linalg.norm(tauT - CT) / np.linalg.norm(CT) < 2e-2
    inc_vds = tauT[0, 1] - tau0[0, 1]
    inc_ode = CT[0, 1] - tau0[0, 1]
    assert inc_ode > 0.08
    assert inc_vds == pytest.approx(inc_ode, rel=1e-2)


def test_exact_dumbbell_moment_values_at_t01():
    # The closed form C_11 = 1 + 2(1 - (1+t)e^{-t}), C_12 = 1 - e^{-t} from C(0) = I
    # (shear rate 1, zeta = 4, H = kT = 1) evaluated by the affine ODE solution.
    import scipy.linalg
    G = wl.shear_gradient(1.0)
    L = (np.kron(G, np.eye(3)) + np.kron(np.eye(3), G)) - np.eye(9)
    c = np.eye(3).reshape(-1)
    t = 0.1
    E = scipy.linalg.expm(L * t)
    C = (E @ np.eye(3).reshape(-1) + np.linalg.solve(L, (E - np.eye(9)) @ c)).reshape(3, 3)
    assert C[0, 0] == pytest.approx(1 + 2 * (1 - (1 + t) * math.exp(-t)), rel=1e-12)
    assert C[0, 1] == pytest.approx(1 - math.exp(-t), rel=1e-12)
    assert C[1, 1] == pytest.approx(1.0, rel=1e-12)


def test_gaussian_ansatz_equilibrium_variance():
    # For a Gaussian particle cloud of variance s^2 the virial identity gives
    # <x . b> = -s^2 (s^2 + 2h^2)/(s^2 + h^2)^2 per component, so the dumbbell's
    # stationary variance solves (s^2 + h^2)^2 = (kT/H)(s^2 + 2h^2).
    rng = np.random.default_rng(13)
    # (continuum statement: finite-P corrections shrink as P h^D grows)
    P, h, s2 = 3000, 0.8, 0.8
    x = rng.standard_normal((P, 3)) * math.sqrt(s2)
    _, t1, t2 = vds.brownian_terms(x, vds.uniform_weights(P), h, threads=4)
    xb = (x * (t1 + t2)).sum(1).mean() / 3
    assert xb == pytest.approx(-s2 * (s2 + 2 * h * h) / (s2 + h * h) ** 2, rel=1e-2)


@pytest.mark.slow
def test_paper_equilibrium_stress_underestimate_at_median_bandwidth():
    # Section 3.2: 2-bead, no flow, P = 1000, median-rule h: the diagonal stress
    # settles about 8% below n (N-1) kT.
    gold = GOLDEN["equilibrium_diag_stress_underestimate"]
    P = 1000
    q = wl.gaussian_bonds(31, 1, P, 1.0)
    h = vds.median_bandwidth(q)
    prob = vds.Problem(nb=1, h=h, dt=0.02)
    w = vds.uniform_weights(P)
    q, _ = vds.run(q, w, prob, 150, scheme="explicit", threads=4)
    under = 1.0 - np.trace(vds.stress(q, w, prob)) / 3.0
    assert abs(under - gold["value"]) <= gold["tolerance"]


def test_median_bandwidth_two_particles():
    # ordered pairs {0, 0, d, d}: median d/2, h = (d/2)/sqrt(2 log 2)
    q = np.zeros((1, 2, 3)); q[0, 1] = [3.0, 4.0, 0.0]
    assert vds.median_bandwidth(q) == pytest.approx(2.5 / math.sqrt(2 * math.log(2)), rel=1e-14)


def test_free_energy_nonincreasing_without_flow_implicit():
    # kappa = 0: the implicit step is the proximal step of F_h, so F_h cannot rise
    P = 150
    q = wl.gaussian_bonds(41, 2, P, 1.0 / 3.0) * 1.7
    prob = vds.Problem(nb=2, h=0.5, dt=5e-3)
    w = vds.uniform_weights(P)
    F = [vds.free_energy(q, w, prob)]
    for _ in range(6):
        q, _ = vds.step_implicit(q, w, prob)
        F.append(vds.free_energy(q, w, prob))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(F, F[1:]))
    assert F[-1] < F[0]


def test_energy_law_rate_matches_work_minus_dissipation():
    # dF_h/dt = W - D along the exact flow: a small explicit step sees
    # (F+ - F)/dt = W - D + O(dt)
    P = 120
    q = wl.gaussian_bonds(43, 3, P, 1.0 / 3.0)
    prob = vds.Problem(nb=3, h=0.4, dt=1e-5, G=wl.shear_gradient(2.0))
    w = vds.uniform_weights(P)
    F0 = vds.free_energy(q, w, prob)
    D0, W0 = vds.dissipation_and_work(q, w, prob)
    q1 = vds.step_explicit(q, w, prob)
    F1 = vds.free_energy(q1, w, prob)
    assert (F1 - F0) / prob.dt == pytest.approx(W0 - D0, rel=1e-3)
    assert D0 > 0


def test_explicit_and_implicit_agree_to_first_order():
    P = 100
    cfg = wl.chain4_shear(P=P, seed=44)
    prob = vds.problem_from(cfg)
    w = vds.uniform_weights(P)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        prob.dt = dt
        n = int(round(0.02 / dt))
        qe, _ = vds.run(cfg["q0"], w, prob, n, scheme="explicit")
        qi, _ = vds.run(cfg["q0"], w, prob, n, scheme="implicit")
        errs.append(np.linalg.norm(qe - qi) / np.linalg.norm(qi))
    # first order: halving dt halves the gap
    assert errs[1] / errs[0] == pytest.approx(0.5, abs=0.08)
    assert errs[2] / errs[1] == pytest.approx(0.5, abs=0.08)


def test_picard_fixed_point_solves_implicit_equation():
    P = 80
    cfg = wl.chain4_shear(P=P, seed=45)
    prob = vds.problem_from(cfg)
    w = vds.uniform_weights(P)
    q = cfg["q0"]
    qp, m = vds.step_implicit(q, w, prob)
    assert 2 <= m <= 8
    # residual of (q+ - q)/dt - G q(t) + (1/zeta)(A (x) I) g(q+) = 0
    g, _ = vds.thermo_force(qp, w, prob)
    res = (qp - q) / prob.dt - vds.flow_term(q, prob) + vds.rouse_apply(vds.rouse_matrix(3), g) / prob.zeta
    assert np.abs(res).max() < 1e-9


def test_density_at_integrates_to_one_in_1d_like_case():
    # f_h(y) for one particle is the normalised Gaussian: f(q_0) = (2 pi h^2)^(-D/2)
    q = np.zeros((1, 1, 3))
    f = vds.density_at(np.zeros((1, 3)), q, np.ones(1), 0.5)
    assert f[0] == pytest.approx((2 * math.pi * 0.25) ** -1.5, rel=1e-14)
