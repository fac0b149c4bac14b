"""GPU parity with the FP64 oracle at the full sizes of the named workloads,
through the C ABI, with the default (FP32) pair kernel:

* 3D Hookean dumbbell, P = 2000, h = 0.3, shear rate 1: the whole run of 100
  implicit steps (Appendix A's implicit scheme), compared every 20 steps and
  at t_end;
* 4-bead chain, P = 20000, D = 9, h = 0.4: the velocity and one implicit
  step on all rows;
* the POD-reduced chain, P = 20000, R = 180 (and R = 60, 120): the Brownian
  operators X^B1 and X^B2 of Section 2.4 against the oracle's factored form
  evaluated one block of kernel-matrix rows at a time;
* the stress history of the reduced run (one entry per output interval).

Tolerances (FP32 GPU against FP64 oracle on the same FP32 inputs): state
relative 2-norm 1e-5, stress relative Frobenius 1e-4, reduced operators 1e-4
(as in the other parity tests).  Per-row bound on the velocity:
||v_gpu - v_oracle||_I / max(||v_oracle||_I, ||(1/zeta)(A (x) I) grad Psi||_I)
<= 1e-4.  Derivation: each row's kernel sums are FP32 within groups of 128
columns (relative rounding below 128 * 2^-24 ~ 8e-6 in the worst case) and
FP64 beyond; the difference x_I S_I - M_I can cancel by up to an order of
magnitude, and the exponent carries |t| 2^-24 with |t| up to ~20 for the pairs
that matter, so a single row can carry up to ~1e-4 while the 2-norm over all
rows stays at the 1e-5 the scheme is held to.
"""
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import pod as opod
from oracle import rom as orom
from oracle import vds as ovds

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))


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


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _rows(a):
    """Per-particle 2-norm over bonds and components of a [nb][P][3] array."""
    return np.sqrt((a ** 2).sum(axis=(0, 2)))


def test_dumbbell_full_run_of_100_implicit_steps_matches_oracle(lib):
    cfg = wl.dumbbell_shear()  # P = 2000, D = 3, h = 0.3, 100 steps
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    qo = wl.f32_as_f64(q32)
    qg = _dev(q32)
    ctx = lib.Context(1, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme="implicit", poison=True)
    done = 0
    while done < cfg["steps"]:
        n = 20
        _say(f"dumbbell P=2000: implicit steps {done}..{done + n} (GPU, one queued call; oracle)")
        d = ctx.step(qg, nsteps=n)
        for _ in range(n):
            qo, _ = ovds.step_implicit(qo, w, prob, threads=THREADS)
        done += n
        assert d["steps"] == n
        assert _rel(_np(qg), qo) < 1e-5, done
        tau_o = ovds.stress(qo, w, prob)
        assert np.linalg.norm(d["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4, done
    assert done == 100


def test_chain4_full_size_velocity_and_implicit_step_on_every_row(lib):
    cfg = wl.chain4_shear()  # P = 20000, D = 9, h = 0.4
    prob = ovds.problem_from(cfg)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    q32 = wl.to_f32(cfg["q0"])
    q0 = wl.f32_as_f64(q32)
    ctx = lib.Context(3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit", poison=True)
    # the velocity of eq. model_DymRepPar on all 20000 rows
    _say("chain4 P=20000: velocity on the GPU and of the oracle on every row")
    v = _np(ctx.velocity(_dev(q32)))
    v_o = ovds.velocity(q0, w, prob, threads=THREADS)
    spring = ovds.rouse_apply(ovds.rouse_matrix(3), ovds.grad_potential(q0, prob)) / prob.zeta
    assert np.linalg.norm(v - v_o) / max(np.linalg.norm(v_o), np.linalg.norm(spring)) < 1e-5
    assert (_rows(v - v_o) / np.maximum(_rows(v_o), _rows(spring))).max() < 1e-4
    # one implicit step on all rows
    qg = _dev(q32)
    _say("chain4 P=20000: one implicit step on the GPU")
    d = ctx.step(qg)
    _say(f"chain4 P=20000: one implicit step of the oracle on {THREADS} threads")
    qo, m = ovds.step_implicit(q0, w, prob, threads=THREADS)
    qgn = _np(qg)
    assert _rel(qgn, qo) < 1e-5
    # per row, the increment q+ - q against the oracle's: the velocity's per-row
    # bound (times dt) plus two FP32 units in the last place of q+, since the
    # stored state itself is rounded to FP32 (2^-24 |q| is ~2e-5 of a step's
    # increment here, so an increment cannot be compared more closely)
    dg, do = qgn - q0, qo - q0
    allow = 1e-4 * np.maximum(_rows(do), prob.dt * _rows(spring)) + 2.0 ** -22 * _rows(qo)
    assert (_rows(dg - do) <= allow).all()
    tau_o = ovds.stress(qo, w, prob)
    assert np.linalg.norm(d["tau"] - tau_o) / np.linalg.norm(tau_o) < 1e-4
    assert 1 <= d["last_iters"] <= m


@pytest.fixture(scope="module")
def chain4_snapshots(lib):
    # 61 states of the 4-bead chain's own trajectory (P = 20000), the POD input
    cfg = wl.chain4_shear()
    P, nb = cfg["P"], 3
    ctx = lib.Context(nb, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit", poison=True)
    import torch
    q = _dev(cfg["q0"])
    snaps = [q.clone()]
    _say("chain4 P=20000: 60 implicit steps for the POD snapshots (GPU)")
    for _ in range(60):
        ctx.step(q, nsteps=1)
        snaps.append(q.clone())
    X = torch.stack(snaps).reshape(61 * nb, 3 * P).contiguous()
    return cfg, ctx, snaps, X


# R = 180 is the POD-reduced chain; on the 256 compute units of an MI355X the
# kernel-GEMM takes 4 column blocks of 32 per workgroup there, 2 at R = 60 and
# 3 at R = 120 (P = 300 in test_gpu_pod_rom.py takes 1)
@pytest.mark.parametrize("R", [180, 60, 120])
def test_reduced_operators_at_full_size_match_row_blocked_oracle(lib, chain4_snapshots, R):
    # the POD-reduced chain: P = 20000 (3P = 60000), operators at the
    # reconstruction of a state of the chain's own trajectory
    cfg, ctx, snaps, X = chain4_snapshots
    P = cfg["P"]
    _say(f"POD basis chain4 P=20000 R={R} from 61 snapshots (GPU)")
    U, _ = ctx.pod_basis(X, R)
    p = ctx.pod_project(U, snaps[30])
    rom = lib.Rom(ctx, U)
    _, XB1, XB2 = (_np(t) for t in rom.operators(p))
    Uf = _np(U).T                                   # 3P x R
    qt = opod.reconstruct(Uf, _np(p), P)
    _say(f"row-blocked oracle operators P=20000 R={R} on {THREADS} threads")
    XB1_o, XB2_o = orom.brownian_rows(Uf, qt, ovds.uniform_weights(P), cfg["h"], threads=THREADS)
    assert _rel(XB1, XB1_o) < 1e-4
    assert _rel(XB2, XB2_o) < 1e-4


def test_reduced_run_stress_history_matches_oracle(lib):
    # vds_rom_run with output_every: one stress per output interval (the last
    # one after the final step), against the oracle's reduced run sampled at
    # the same steps; output_every = 0 gives only the final stress
    P, R, steps, every, out = 300, 24, 47, 10, 5
    rng = np.random.default_rng(31)
    U, _ = np.linalg.qr(rng.standard_normal((3 * P, R)))
    U32 = wl.to_f32(U.T)
    Uf = U32.astype(np.float64).T
    q = wl.gaussian_bonds(31, 3, P, 1 / 3)
    p32 = wl.to_f32(opod.project(Uf, wl.f32_as_f64(wl.to_f32(q))))
    prob = ovds.Problem(nb=3, h=0.5, dt=1e-3, G=wl.shear_gradient(1.0))
    ctx = lib.Context(3, P, prob.h, G=prob.G, dt=prob.dt, scheme="explicit", poison=True)
    rom = lib.Rom(ctx, _dev(U32))
    _say("reduced run P=300 R=24 with a stress history")
    p = _dev(p32)
    hist = rom.run(p, nsteps=steps, freeze_every=every, output_every=out)
    assert hist.shape == (-(-steps // out), 3, 3)
    w = ovds.uniform_weights(P)
    want = {}
    q0 = opod.reconstruct(Uf, p32.astype(np.float64), P)

    def record(s, pp):
        if s % out == 0 or s == steps:
            want[s] = orom.reduced_stress(Uf, pp, w, prob, P)

    orom.rom_run(Uf, q0, w, prob, steps, every, callback=record)
    keys = sorted(want)
    assert len(keys) == hist.shape[0]
    for i, s in enumerate(keys):
        assert np.linalg.norm(hist[i] - want[s]) / np.linalg.norm(want[s]) < 1e-4, s
    # the final entry is the stress of the final state, as output_every = 0 gives it
    p2 = _dev(p32)
    tau_final = rom.run(p2, nsteps=steps, freeze_every=every)
    assert np.array_equal(tau_final, hist[-1])
    with pytest.raises(lib.VDSError):
        rom.run(_dev(p32), nsteps=3, freeze_every=1, output_every=-1)
