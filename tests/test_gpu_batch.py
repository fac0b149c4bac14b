"""GPU parity of the batched ensembles (include/vds_batch.h) against the FP64
oracle run per ensemble, and of the captured-graph step against eager launches.

Tolerances: states relative 1e-5 (float32 vs float64 oracle on the same float32
inputs, a few explicit steps); per-ensemble stress relative Frobenius 1e-4;
graph replays bitwise equal to eager launches (same kernels, fixed reduction
order).  Every pair implementation is covered: the FP32 32x32 form (the
default), the FP32 16x16 form and the FP16-split forms."""
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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _small_batch():
    P = np.array([17, 300, 1000, 257, 2000, 64])
    rate = np.array([0.1, 1.0, 3.0, 10.0, 0.5, 2.0])
    h = 0.4 * (P / 2000.0) ** (-1.0 / 13)
    G = np.stack([wl.shear_gradient(r) for r in rate])
    states = [wl.gaussian_bonds(50 + e, 3, int(P[e]), 1 / 3) for e in range(len(P))]
    return P, h, G, states


def _oracle_steps(q, P, h, G, nsteps):
    prob = ovds.Problem(nb=3, h=h, dt=1e-3, G=G)
    w = ovds.uniform_weights(P)
    for _ in range(nsteps):
        q = ovds.step_explicit(q, w, prob, threads=8)
    return q, ovds.stress(q, w, prob)


IMPLS = (4, 0, 2, 3)  # FP32 32x32 and 16x16 MFMA, the two FP16-split forms


@pytest.mark.parametrize("impl", IMPLS)
def test_batch_matches_oracle_per_ensemble(lib, impl):
    import torch
    P, h, G, states = _small_batch()
    b = lib.Batch(P, h, G, poison=True)
    b.set_tuning(2, 1024, impl=impl)
    q = b.pack([torch.from_numpy(wl.to_f32(s)).cuda() for s in states])
    tau = b.step(q, nsteps=3, stress=True)
    out = b.unpack(q)
    for e in range(len(P)):
        _say(f"impl {impl} ensemble {e} P={P[e]}")
        qo, tau_o = _oracle_steps(wl.f32_as_f64(wl.to_f32(states[e])), int(P[e]), h[e], G[e], 3)
        assert _rel(out[e].cpu().numpy(), qo) < 1e-5, e
        assert np.linalg.norm(tau[e] - tau_o) / np.linalg.norm(tau_o) < 1e-4, e


@pytest.mark.parametrize("impl", IMPLS)
def test_graph_replays_equal_eager_launches(lib, impl):
    import torch
    P, h, G, states = _small_batch()
    b = lib.Batch(P, h, G, poison=True)
    q0 = b.pack([torch.from_numpy(wl.to_f32(s)).cuda() for s in states])
    _say(f"graph replays impl {impl}")
    b.set_tuning(2, 512, use_graph=False, impl=impl)
    qe = q0.clone()
    eager = []
    for _ in range(4):
        b.step(qe, nsteps=1)
        eager.append(qe.clone())
    b.set_tuning(2, 512, use_graph=True)
    qg = q0.clone()
    for s in range(4):
        b.step(qg, nsteps=1)
        torch.cuda.synchronize()
        _ = (qg * 2).sum().item()          # eager work between replays
        assert torch.equal(qg, eager[s]), s


def test_tunings_agree_and_autotune_is_valid(lib):
    import torch
    P, h, G, states = _small_batch()
    b = lib.Batch(P, h, G, poison=True)
    q0 = b.pack([torch.from_numpy(wl.to_f32(s)).cuda() for s in states])
    refs = {}
    for impl in IMPLS:
        for rb in ((1, 2) if impl == 4 else (1, 2, 4)):
            for grid in (7, 256, 2048):
                _say(f"batch tuning impl {impl} rb {rb} grid {grid}")
                b.set_tuning(rb, grid, impl=impl)
                q = q0.clone()
                b.step(q, nsteps=2)
                r = q.cpu().numpy()
                ref = refs.setdefault(impl, r)
                assert np.array_equal(r, ref), (impl, rb, grid)   # one split: identical arithmetic
    # the implementations agree with each other to the parity tolerance
    for impl in IMPLS[1:]:
        assert _rel(refs[impl], refs[IMPLS[0]].astype(np.float64)) < 1e-5, impl
    t = b.autotune(q0)
    assert t["impl"] in IMPLS and t["rows_per_wave"] in (1, 2, 4) and t["grid"] >= 1


def test_batch_matches_single_ensemble_contexts(lib):
    import torch
    P, h, G, states = _small_batch()
    b = lib.Batch(P, h, G, poison=True)
    q = b.pack([torch.from_numpy(wl.to_f32(s)).cuda() for s in states])
    b.step(q, nsteps=2)
    out = b.unpack(q)
    for e in (1, 4):
        ctx = lib.Context(3, int(P[e]), h[e], G=G[e], dt=1e-3, scheme="explicit", poison=True)
        qs = torch.from_numpy(wl.to_f32(states[e])).cuda()
        ctx.step(qs, nsteps=2)
        assert _rel(out[e].cpu().numpy(), qs.cpu().numpy().astype(np.float64)) < 1e-5


def test_full_size_512_ensembles_sampled_vs_oracle(lib):
    # the 512-ensemble workload (P_b in [2000, 16000], shear rates log-uniform in
    # [0.1, 10], h_b = 0.4 (P_b/20000)^(-1/13)); one step, three sampled ensembles
    import torch
    ens = wl.ensembles()
    _say("batch 512 ensembles, total P", int(ens["P"].sum()))
    G = np.stack([wl.shear_gradient(r) for r in ens["rate"]])
    b = lib.Batch(ens["P"], ens["h"], G)
    states = [wl.ensemble_state(ens, e) for e in range(ens["n_ens"])]
    q = b.pack([torch.from_numpy(wl.to_f32(s)).cuda() for s in states])
    b.autotune(q)
    tau = b.step(q, nsteps=1, stress=True)
    out = b.unpack(q)
    order = np.argsort(ens["P"])
    for e in (int(order[0]), int(order[1]), int(order[len(order) // 2])):
        _say(f"sampled ensemble {e} P={ens['P'][e]}")
        qo, tau_o = _oracle_steps(wl.f32_as_f64(wl.to_f32(states[e])), int(ens["P"][e]), ens["h"][e], G[e], 1)
        assert _rel(out[e].cpu().numpy(), qo) < 1e-5, e
        assert np.linalg.norm(tau[e] - tau_o) / np.linalg.norm(tau_o) < 1e-4, e
