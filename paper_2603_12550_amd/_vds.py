"""ctypes binding of libvds.so: the C ABI of include/vds.h, one Python function
per C entry point with the same name, plus a small `Context` convenience class.

Argument marshalling only: tensors pass their device pointers, host structs are
ctypes mirrors of the C ones.  Every step of the computation runs in the HIP
library; if it is not built this module raises at import time.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvds.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_12550_amd/build.py "
                      "(or __graft_entry__.build()); there is no CPU fallback")
_lib = C.CDLL(LIB_PATH)

VDS_OK, VDS_ERR_ARG, VDS_ERR_HIP, VDS_ERR_NOMEM, VDS_ERR_NOT_CONVERGED, VDS_ERR_STATE = range(6)
VDS_HOOKEAN, VDS_FENE = 0, 1
VDS_EXPLICIT, VDS_IMPLICIT = 0, 1
VDS_PAIR_MFMA, VDS_PAIR_VALU, VDS_PAIR_MFMA_F16X2, VDS_PAIR_MFMA_F16X2_ALL, VDS_PAIR_MFMA32 = 0, 1, 2, 3, 4
VDS_TIMER_PAIR, VDS_TIMER_GEMM, VDS_TIMER_KGEMM, VDS_TIMER_PROJ = range(4)
STATUS_NAMES = {0: "VDS_OK", 1: "VDS_ERR_ARG", 2: "VDS_ERR_HIP", 3: "VDS_ERR_NOMEM",
                4: "VDS_ERR_NOT_CONVERGED", 5: "VDS_ERR_STATE"}


class vds_problem(C.Structure):
    _fields_ = [("nb", C.c_int32), ("potential", C.c_int32), ("P", C.c_int64), ("kT", C.c_double),
                ("zeta", C.c_double), ("n", C.c_double), ("h", C.c_double), ("dt", C.c_double),
                ("G", C.c_double * 9), ("b_max", C.c_double), ("scheme", C.c_int32),
                ("picard_max", C.c_int32), ("picard_rtol", C.c_double), ("picard_batch", C.c_int32),
                ("picard_predictor", C.c_int32)]


class vds_diag(C.Structure):
    _fields_ = [("steps", C.c_int32), ("iters", C.c_int32), ("last_iters", C.c_int32),
                ("energy_valid", C.c_int32), ("resid", C.c_double), ("F", C.c_double),
                ("dissipation", C.c_double), ("work", C.c_double), ("tau", C.c_double * 9)]

    def as_dict(self):
        return dict(steps=self.steps, iters=self.iters, last_iters=self.last_iters,
                    energy_valid=self.energy_valid, resid=self.resid, F=self.F,
                    dissipation=self.dissipation, work=self.work,
                    tau=np.array(self.tau[:]).reshape(3, 3))


class vds_tuning(C.Structure):
    _fields_ = [("impl", C.c_int32), ("rows_per_wave", C.c_int32), ("col_splits", C.c_int32),
                ("reserved", C.c_int32)]


_P = C.c_void_p
_sigs = {
    "vds_create": ([C.POINTER(vds_problem), C.POINTER(C.c_double), _P, C.POINTER(_P)], C.c_int),
    "vds_destroy": ([_P], None),
    "vds_workspace_bytes": ([C.POINTER(vds_problem)], C.c_size_t),
    "vds_bind_workspace": ([_P, _P, C.c_size_t], C.c_int),
    "vds_last_error": ([_P], C.c_char_p),
    "vds_set_tuning": ([_P, C.POINTER(vds_tuning)], C.c_int),
    "vds_get_tuning": ([_P, C.POINTER(vds_tuning)], C.c_int),
    "vds_autotune": ([_P, _P, _P], C.c_int),
    "vds_pair_sums": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "vds_pair_sums_noalloc": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "vds_velocity": ([_P, _P, _P, _P, C.POINTER(vds_diag)], C.c_int),
    "vds_step": ([_P, _P, _P, C.c_int32, C.POINTER(vds_diag)], C.c_int),
    "vds_stress": ([_P, _P, _P, C.POINTER(C.c_double)], C.c_int),
    "vds_energy": ([_P, _P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "vds_density_at": ([_P, _P, _P, _P, C.c_int64, _P], C.c_int),
    "vds_median_bandwidth": ([_P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "vds_timing_enable": ([_P, C.c_int32], C.c_int),
    "vds_timing_read": ([_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)], C.c_int),
}
_sigs.update({
    "vds_pod_workspace_bytes": ([C.c_int64, C.c_int32, C.c_int32], C.c_size_t),
    "vds_pod_gram": ([_P, _P, C.c_int64, C.c_int32, _P, _P, C.c_size_t], C.c_int),
    "vds_pod_basis": ([_P, _P, C.c_int64, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double), _P, C.c_size_t], C.c_int),
    "vds_pod_map_workspace_bytes": ([C.POINTER(vds_problem), C.c_int32], C.c_size_t),
    "vds_pod_project": ([_P, _P, C.c_int32, _P, _P, _P, C.c_size_t], C.c_int),
    "vds_pod_reconstruct": ([_P, _P, C.c_int32, _P, _P, _P, C.c_size_t], C.c_int),
    "vds_rom_workspace_bytes": ([C.POINTER(vds_problem), C.c_int32], C.c_size_t),
    "vds_rom_create": ([_P, _P, C.c_int32, _P, C.c_size_t, C.POINTER(_P)], C.c_int),
    "vds_rom_destroy": ([_P], None),
    "vds_rom_operators": ([_P, _P, _P, _P, _P], C.c_int),
    "vds_rom_run": ([_P, _P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "vds_rom_run_midpoint": ([_P, _P, C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "vds_rom_run_extrapolated": ([_P, _P, C.c_int32, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "vds_rom_stress": ([_P, _P, C.POINTER(C.c_double)], C.c_int),
})


class vds_rom_window_stats(C.Structure):
    _fields_ = [("windows", C.c_int32), ("rejected", C.c_int32), ("truncated", C.c_int32), ("recorded", C.c_int32),
                ("t_reached", C.c_double), ("max_energy_gap", C.c_double)]


_sigs.update({
    "vds_rom_exact_workspace_bytes": ([_P, C.c_int32], C.c_size_t),
    "vds_rom_run_exact": ([_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_double), C.c_int32,
                           _P, C.c_size_t, C.POINTER(C.c_double), C.POINTER(vds_rom_window_stats)], C.c_int),
})
_sigs.update({
    "vds_batch_workspace_bytes": ([C.c_int32, C.POINTER(C.c_int64), C.c_int32], C.c_size_t),
    "vds_batch_create": ([C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double),
                          C.POINTER(vds_problem), C.POINTER(C.c_double), _P, C.POINTER(_P)], C.c_int),
    "vds_batch_bind_workspace": ([_P, _P, C.c_size_t], C.c_int),
    "vds_batch_destroy": ([_P], None),
    "vds_batch_last_error": ([_P], C.c_char_p),
    "vds_batch_state_offset": ([_P, C.c_int32], C.c_int64),
    "vds_batch_set_tuning": ([_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "vds_batch_get_tuning": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32)], C.c_int),
    "vds_batch_autotune": ([_P, _P], C.c_int),
    "vds_batch_step": ([_P, _P, C.c_int32, C.POINTER(C.c_double)], C.c_int),
})
class vds_mlp_rollout(C.Structure):
    _fields_ = [("steps", C.c_int32), ("checks", C.c_int32), ("fallbacks", C.c_int32), ("reserved", C.c_int32),
                ("max_resid", C.c_double), ("max_energy_gap", C.c_double), ("tau", C.c_double * 9)]


_sigs.update({
    "vds_mlp_workspace_bytes": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32], C.c_size_t),
    "vds_mlp_create": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.POINTER(_P)], C.c_int),
    "vds_mlp_bind_workspace": ([_P, _P, C.c_size_t], C.c_int),
    "vds_mlp_destroy": ([_P], None),
    "vds_mlp_last_error": ([_P], C.c_char_p),
    "vds_mlp_param_count": ([_P], C.c_int64),
    "vds_mlp_set_params": ([_P, _P], C.c_int),
    "vds_mlp_get_params": ([_P, _P], C.c_int),
    "vds_mlp_get_grads": ([_P, _P], C.c_int),
    "vds_mlp_forward": ([_P, _P, C.c_int32, _P, C.c_int32], C.c_int),
    "vds_mlp_predict_steps": ([_P, _P, C.c_float, C.c_int32], C.c_int),
    "vds_mlp_set_input_noise": ([_P, C.c_float, C.c_uint64], C.c_int),
    "vds_mlp_loss_grad": ([_P, _P, _P, C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "vds_mlp_adam_step": ([_P, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
    "vds_mlp_train_epoch": ([_P, _P, _P, C.c_int32, C.c_int32, C.c_float, _P, C.POINTER(C.c_double)], C.c_int),
    "vds_mlp_set_scaling": ([_P, _P, _P, _P, _P], C.c_int),
    "vds_mlp_fit_scaling": ([_P, _P, _P, C.c_int32], C.c_int),
    "vds_mlp_make_pairs": ([_P, _P, C.c_int32, C.c_float, _P, _P], C.c_int),
    "vds_mlp_rollout_workspace_bytes": ([C.POINTER(vds_problem), C.c_int32], C.c_size_t),
    "vds_mlp_rollout_run": ([_P, _P, _P, C.c_int32, _P, C.c_float, C.c_int32, C.c_int32, C.c_double, C.c_double,
                             _P, C.c_size_t, C.POINTER(vds_mlp_rollout)], C.c_int),
})
for _name, (_args, _ret) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _ret

EXPORTED = tuple(_sigs)


class VDSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _check(status, ctx=None):
    if status != VDS_OK:
        msg = _lib.vds_last_error(ctx)
        raise VDSError(status, msg.decode() if msg else "")


def make_problem(nb, P, h, dt=1e-3, kT=1.0, zeta=4.0, n=1.0, G=None, potential="hookean", b_max=0.0,
                 scheme="implicit", picard_max=50, picard_rtol=1e-6, picard_batch=3,
                 picard_predictor=0) -> vds_problem:
    pr = vds_problem()
    pr.nb, pr.P, pr.h, pr.dt, pr.kT, pr.zeta, pr.n = int(nb), int(P), float(h), float(dt), float(kT), float(zeta), float(n)
    G = np.zeros((3, 3)) if G is None else np.asarray(G, dtype=np.float64).reshape(3, 3)
    for i, v in enumerate(G.reshape(-1)):
        pr.G[i] = float(v)
    pr.potential = VDS_FENE if potential == "fene" else VDS_HOOKEAN
    pr.b_max = float(b_max)
    pr.scheme = VDS_IMPLICIT if scheme == "implicit" else VDS_EXPLICIT
    pr.picard_max, pr.picard_rtol, pr.picard_batch = int(picard_max), float(picard_rtol), int(picard_batch)
    pr.picard_predictor = int(picard_predictor)
    return pr


class Context:
    """One problem on one HIP stream, with a torch-allocated workspace."""

    def __init__(self, nb, P, h, H=None, stream=None, device="cuda", poison=False, **kw):
        self.nb, self.P, self.D = int(nb), int(P), 3 * int(nb)
        self.device = torch.device(device)
        self.prob = make_problem(nb, P, h, **kw)
        H = np.ones(self.nb) if H is None else np.asarray(H, dtype=np.float64)
        self._H = (C.c_double * self.nb)(*[float(v) for v in H])
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        _check(_lib.vds_create(C.byref(self.prob), self._H, C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        nbytes = _lib.vds_workspace_bytes(C.byref(self.prob))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if poison:  # NaN-fill: any read of workspace the library did not write shows up
            self.ws.fill_(255)
        _check(_lib.vds_bind_workspace(self.ctx, _ptr(self.ws), nbytes), self.ctx)

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "ctx", None) and _lib is not None:
            _lib.vds_destroy(self.ctx)
            self.ctx = None

    # -- tuning / timing --
    def set_tuning(self, impl=VDS_PAIR_MFMA32, rows_per_wave=2, col_splits=4):
        t = vds_tuning(impl, rows_per_wave, col_splits, 0)
        _check(_lib.vds_set_tuning(self.ctx, C.byref(t)), self.ctx)

    def get_tuning(self):
        t = vds_tuning()
        _check(_lib.vds_get_tuning(self.ctx, C.byref(t)), self.ctx)
        return dict(impl=t.impl, rows_per_wave=t.rows_per_wave, col_splits=t.col_splits)

    def autotune(self, q, w=None):
        _check(_lib.vds_autotune(self.ctx, _ptr(q), _ptr(w)), self.ctx)
        return self.get_tuning()

    def timing_enable(self, on=True, stride=1):
        """Event timing of every `stride`-th launch of each timed kernel."""
        _check(_lib.vds_timing_enable(self.ctx, int(stride) if on else 0), self.ctx)

    def timing_read(self, which=VDS_TIMER_PAIR):
        ms, n, work = C.c_double(), C.c_int64(), C.c_double()
        _check(_lib.vds_timing_read(self.ctx, which, C.byref(ms), C.byref(n), C.byref(work)), self.ctx)
        return dict(ms=ms.value, launches=n.value, work=work.value)

    # -- scheme --
    def _state(self):
        return torch.empty((self.nb, self.P, 3), dtype=torch.float32, device=self.device)

    def pair_sums(self, q, w=None):
        S = torch.empty(self.P, dtype=torch.float32, device=self.device)
        t1, t2 = self._state(), self._state()
        _check(_lib.vds_pair_sums(self.ctx, _ptr(q), _ptr(w), _ptr(S), _ptr(t1), _ptr(t2)), self.ctx)
        return S, t1, t2

    def velocity(self, q, w=None, diag=False):
        v = self._state()
        d = vds_diag()
        _check(_lib.vds_velocity(self.ctx, _ptr(q), _ptr(w), _ptr(v), C.byref(d) if diag else None), self.ctx)
        return (v, d.as_dict()) if diag else v

    def step(self, q, w=None, nsteps=1):
        d = vds_diag()
        st = _lib.vds_step(self.ctx, _ptr(q), _ptr(w), int(nsteps), C.byref(d))
        _check(st, self.ctx)
        return d.as_dict()

    def stress(self, q, w=None):
        tau = (C.c_double * 9)()
        _check(_lib.vds_stress(self.ctx, _ptr(q), _ptr(w), tau), self.ctx)
        return np.array(tau[:]).reshape(3, 3)

    def energy(self, q, w=None):
        F, Dd, W = C.c_double(), C.c_double(), C.c_double()
        _check(_lib.vds_energy(self.ctx, _ptr(q), _ptr(w), C.byref(F), C.byref(Dd), C.byref(W)), self.ctx)
        return F.value, Dd.value, W.value

    # -- POD (Sections 1.3, 2.3, 3.1) --
    def _pod_ws(self, m, ncols, R):
        n = _lib.vds_pod_workspace_bytes(int(m), int(ncols), int(R))
        if n == 0:
            raise VDSError(VDS_ERR_ARG, "invalid POD sizes")
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def pod_gram(self, X):
        """X: tensor (ncols, m) holding the column-major m x ncols snapshot matrix."""
        ncols, m = X.shape
        G = torch.empty((ncols, ncols), dtype=torch.float32, device=self.device)
        ws = self._pod_ws(m, ncols, 1)
        _check(_lib.vds_pod_gram(self.ctx, _ptr(X), m, ncols, _ptr(G), _ptr(ws), ws.numel()), self.ctx)
        return G

    def pod_basis(self, X, R):
        """Returns U as a tensor (R, m) (column-major m x R) and all eigenvalues, descending."""
        ncols, m = X.shape
        U = torch.empty((R, m), dtype=torch.float32, device=self.device)
        eig = (C.c_double * ncols)()
        ws = self._pod_ws(m, ncols, R)
        _check(_lib.vds_pod_basis(self.ctx, _ptr(X), m, ncols, int(R), _ptr(U), eig, _ptr(ws), ws.numel()), self.ctx)
        return U, np.array(eig[:])

    def _map_ws(self, R):
        n = _lib.vds_pod_map_workspace_bytes(C.byref(self.prob), int(R))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def pod_project(self, U, q):
        R = U.shape[0]
        p = torch.empty((self.nb, R), dtype=torch.float32, device=self.device)
        ws = self._map_ws(R)
        _check(_lib.vds_pod_project(self.ctx, _ptr(U), R, _ptr(q), _ptr(p), _ptr(ws), ws.numel()), self.ctx)
        return p

    def pod_reconstruct(self, U, p):
        R = U.shape[0]
        q = self._state()
        ws = self._map_ws(R)
        _check(_lib.vds_pod_reconstruct(self.ctx, _ptr(U), R, _ptr(p), _ptr(q), _ptr(ws), ws.numel()), self.ctx)
        return q

    def median_bandwidth(self, q):
        """(med, h) of the median rule (eq. model_bandwidth) for the state q."""
        med, h = C.c_double(), C.c_double()
        _check(_lib.vds_median_bandwidth(self.ctx, _ptr(q), C.byref(med), C.byref(h)), self.ctx)
        return med.value, h.value

    def density_at(self, q, y, w=None):
        y = y.contiguous()
        f = torch.empty(y.shape[0], dtype=torch.float32, device=self.device)
        _check(_lib.vds_density_at(self.ctx, _ptr(q), _ptr(w), _ptr(y), int(y.shape[0]), _ptr(f)), self.ctx)
        return f


class Rom:
    """Galerkin reduced model (Section 2.4) of basis U (tensor (R, 3P)) on a Context."""

    def __init__(self, ctx: Context, U):
        self.ctx, self.U, self.R = ctx, U, int(U.shape[0])
        n = _lib.vds_rom_workspace_bytes(C.byref(ctx.prob), self.R)
        if n == 0:
            raise VDSError(VDS_ERR_ARG, "invalid reduced-model sizes")
        self.ws = torch.empty(n, dtype=torch.uint8, device=ctx.device)
        h = C.c_void_p()
        _check(_lib.vds_rom_create(ctx.ctx, _ptr(U), self.R, _ptr(self.ws), n, C.byref(h)), ctx.ctx)
        self.rom = h

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "rom", None) and _lib is not None:
            _lib.vds_rom_destroy(self.rom)
            self.rom = None

    def operators(self, p):
        R = self.R
        XH, XB1, XB2 = (torch.empty((R, R), dtype=torch.float32, device=self.ctx.device) for _ in range(3))
        _check(_lib.vds_rom_operators(self.rom, _ptr(p), _ptr(XH), _ptr(XB1), _ptr(XB2)), self.ctx.ctx)
        return XH, XB1, XB2

    def run(self, p, nsteps, freeze_every, midpoint=False, output_every=0):
        """Reduced explicit Euler steps; returns the final stress, or with
        output_every >= 1 the stress history (vds_rom_run), shape
        (ceil(nsteps / output_every), 3, 3).  With `midpoint` the operators of
        each window come from its predicted midpoint (vds_rom_run_midpoint),
        with `midpoint="extrapolated"` from the midpoint extrapolated from the
        last two window starts (vds_rom_run_extrapolated)."""
        if midpoint:
            if output_every:
                raise ValueError("the midpoint forms return the final stress only")
            tau = (C.c_double * 9)()
            fn = _lib.vds_rom_run_extrapolated if midpoint == "extrapolated" else _lib.vds_rom_run_midpoint
            _check(fn(self.rom, _ptr(p), int(nsteps), int(freeze_every), tau), self.ctx.ctx)
            return np.array(tau[:]).reshape(3, 3)
        nout = -(-int(nsteps) // int(output_every)) if output_every > 0 else 1
        tau = (C.c_double * (9 * max(1, nout)))()
        _check(_lib.vds_rom_run(self.rom, _ptr(p), int(nsteps), int(freeze_every), int(output_every), tau),
               self.ctx.ctx)
        hist = np.array(tau[:]).reshape(-1, 3, 3)
        return hist if output_every > 0 else hist[0]

    def stress(self, p):
        tau = (C.c_double * 9)()
        _check(_lib.vds_rom_stress(self.rom, _ptr(p), tau), self.ctx.ctx)
        return np.array(tau[:]).reshape(3, 3)

    def run_exact(self, p, nsteps, freeze_every, adaptive=False, energy_tol=0.1, max_windows=4096):
        """Windows integrated exactly (see vds_rom_run_exact); returns the
        stress, the accepted window lengths and the counts."""
        n = _lib.vds_rom_exact_workspace_bytes(C.byref(self.ctx.prob), self.R)
        if getattr(self, "ws_exact", None) is None or self.ws_exact.numel() < n:
            self.ws_exact = torch.empty(n, dtype=torch.uint8, device=self.ctx.device)
        tau = (C.c_double * 9)()
        win = (C.c_double * max_windows)()
        st = vds_rom_window_stats()
        _check(_lib.vds_rom_run_exact(self.rom, _ptr(p), int(nsteps), int(freeze_every), 1 if adaptive else 0,
                                      float(energy_tol), win, int(max_windows), _ptr(self.ws_exact), n, tau,
                                      C.byref(st)), self.ctx.ctx)
        stats = {f: getattr(st, f) for f, _ in vds_rom_window_stats._fields_}
        return np.array(tau[:]).reshape(3, 3), list(win[:st.recorded]), stats


def _bcheck(status, b=None):
    if status != VDS_OK:
        msg = _lib.vds_batch_last_error(b)
        raise VDSError(status, msg.decode() if msg else "")


class Batch:
    """Independent ensembles advanced together (include/vds_batch.h); the state
    is one packed float32 device tensor of the ensembles' [nb][P_b][3] blocks."""

    def __init__(self, P, h, G, nb=3, H=None, kT=1.0, zeta=4.0, n=1.0, dt=1e-3, potential="hookean", b_max=0.0,
                 stream=None, device="cuda", poison=False):
        self.P = np.asarray(P, dtype=np.int64)
        self.nens, self.nb = len(self.P), int(nb)
        self.device = torch.device(device)
        Parr = (C.c_int64 * self.nens)(*[int(v) for v in self.P])
        harr = (C.c_double * self.nens)(*[float(v) for v in np.asarray(h, dtype=np.float64)])
        Garr = (C.c_double * (9 * self.nens))(*[float(v) for v in np.asarray(G, dtype=np.float64).reshape(-1)])
        H = np.ones(self.nb) if H is None else np.asarray(H, dtype=np.float64)
        Harr = (C.c_double * self.nb)(*[float(v) for v in H])
        common = make_problem(nb, 1, 1.0, dt=dt, kT=kT, zeta=zeta, n=n, potential=potential, b_max=b_max,
                              scheme="explicit")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        b = C.c_void_p()
        _bcheck(_lib.vds_batch_create(self.nens, Parr, harr, Garr, C.byref(common), Harr,
                                      C.c_void_p(self.stream.cuda_stream), C.byref(b)))
        self.b = b
        nbytes = _lib.vds_batch_workspace_bytes(self.nens, Parr, self.nb)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if poison:
            self.ws.fill_(255)
        _bcheck(_lib.vds_batch_bind_workspace(self.b, _ptr(self.ws), nbytes), self.b)
        self.offsets = [int(_lib.vds_batch_state_offset(self.b, e)) for e in range(self.nens + 1)]

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "b", None) and _lib is not None:
            _lib.vds_batch_destroy(self.b)
            self.b = None

    def pack(self, states):
        return torch.cat([s.reshape(-1) for s in states]).contiguous()

    def unpack(self, q):
        return [q[self.offsets[e]:self.offsets[e + 1]].reshape(self.nb, int(self.P[e]), 3) for e in range(self.nens)]

    def set_tuning(self, rows_per_wave=2, grid=1024, use_graph=True, impl=None):
        """impl None keeps the current pair implementation."""
        if impl is None:
            impl = self.get_tuning()["impl"]
        _bcheck(_lib.vds_batch_set_tuning(self.b, int(impl), int(rows_per_wave), int(grid), 1 if use_graph else 0),
                self.b)

    def get_tuning(self):
        im, rb, g, u = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _bcheck(_lib.vds_batch_get_tuning(self.b, C.byref(im), C.byref(rb), C.byref(g), C.byref(u)), self.b)
        return dict(impl=im.value, rows_per_wave=rb.value, grid=g.value, use_graph=u.value)

    def autotune(self, q):
        _bcheck(_lib.vds_batch_autotune(self.b, _ptr(q)), self.b)
        return self.get_tuning()

    def step(self, q, nsteps=1, stress=False):
        tau = (C.c_double * (9 * self.nens))() if stress else None
        _bcheck(_lib.vds_batch_step(self.b, _ptr(q), int(nsteps), tau), self.b)
        return np.array(tau[:]).reshape(self.nens, 3, 3) if stress else None


def _mcheck(status, m=None):
    if status != VDS_OK:
        msg = _lib.vds_mlp_last_error(m)
        raise VDSError(status, msg.decode() if msg else "")


class Mlp:
    """Learned reduced step (include/vds_mlp.h): nin -> width -> width -> nout, SiLU."""

    def __init__(self, nin, width, nout, max_batch, stream=None, device="cuda"):
        self.nin, self.width, self.nout, self.max_batch = int(nin), int(width), int(nout), int(max_batch)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _mcheck(_lib.vds_mlp_create(self.nin, self.width, self.nout, self.max_batch,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.m = h
        n = _lib.vds_mlp_workspace_bytes(self.nin, self.width, self.nout, self.max_batch)
        self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        _mcheck(_lib.vds_mlp_bind_workspace(self.m, _ptr(self.ws), n), self.m)
        self.nparams = int(_lib.vds_mlp_param_count(self.m))

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "m", None) and _lib is not None:
            _lib.vds_mlp_destroy(self.m)
            self.m = None

    def set_params(self, flat):
        _mcheck(_lib.vds_mlp_set_params(self.m, _ptr(flat.contiguous())), self.m)

    def get_params(self):
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _mcheck(_lib.vds_mlp_get_params(self.m, _ptr(out)), self.m)
        return out

    def get_grads(self):
        out = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _mcheck(_lib.vds_mlp_get_grads(self.m, _ptr(out)), self.m)
        return out

    def forward(self, X, bf16=False):
        Y = torch.empty((X.shape[0], self.nout), dtype=torch.float32, device=self.device)
        _mcheck(_lib.vds_mlp_forward(self.m, _ptr(X), int(X.shape[0]), _ptr(Y), 1 if bf16 else 0), self.m)
        return Y

    def set_input_noise(self, sigma, seed=0):
        """Training input noise of sigma increment standard deviations."""
        _mcheck(_lib.vds_mlp_set_input_noise(self.m, float(sigma), int(seed)), self.m)

    def predict_steps(self, p, log_rate, nsteps):
        """nsteps learned steps on the reduced state p (in place)."""
        _mcheck(_lib.vds_mlp_predict_steps(self.m, _ptr(p), float(log_rate), int(nsteps)), self.m)
        return p

    def loss_grad(self, X, T):
        loss = C.c_double()
        _mcheck(_lib.vds_mlp_loss_grad(self.m, _ptr(X), _ptr(T), int(X.shape[0]), C.byref(loss)), self.m)
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _mcheck(_lib.vds_mlp_adam_step(self.m, float(lr), float(beta1), float(beta2), float(eps)), self.m)

    def train_epoch(self, X, T, batch, lr, order=None):
        loss = C.c_double()
        _mcheck(_lib.vds_mlp_train_epoch(self.m, _ptr(X), _ptr(T), int(X.shape[0]), int(batch), float(lr),
                                         _ptr(order), C.byref(loss)), self.m)
        return loss.value

    def fit_scaling(self, X, T):
        _mcheck(_lib.vds_mlp_fit_scaling(self.m, _ptr(X), _ptr(T), int(X.shape[0])), self.m)

    def make_pairs(self, traj, log_rate):
        nt = int(traj.shape[0])
        X = torch.empty((nt - 1, self.nin), dtype=torch.float32, device=self.device)
        T = torch.empty((nt - 1, self.nout), dtype=torch.float32, device=self.device)
        _mcheck(_lib.vds_mlp_make_pairs(self.m, _ptr(traj), nt, float(log_rate), _ptr(X), _ptr(T)), self.m)
        return X, T

    def set_scaling(self, x_shift, x_scale, y_shift, y_scale):
        ts = [t.contiguous() for t in (x_shift, x_scale, y_shift, y_scale)]
        _mcheck(_lib.vds_mlp_set_scaling(self.m, *[_ptr(t) for t in ts]), self.m)

    def rollout(self, ctx, U, p, log_rate, nsteps, check_every, resid_tol, energy_tol):
        R = int(U.shape[0])
        n = _lib.vds_mlp_rollout_workspace_bytes(C.byref(ctx.prob), R)
        ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        st = vds_mlp_rollout()
        _mcheck(_lib.vds_mlp_rollout_run(self.m, ctx.ctx, _ptr(U), R, _ptr(p), float(log_rate), int(nsteps),
                                         int(check_every), float(resid_tol), float(energy_tol), _ptr(ws), n,
                                         C.byref(st)), self.m)
        return dict(steps=st.steps, checks=st.checks, fallbacks=st.fallbacks, max_resid=st.max_resid,
                    max_energy_gap=st.max_energy_gap, tau=np.array(st.tau[:]).reshape(3, 3))


# C names, re-exported for callers who drive the ABI directly
globals().update({name: getattr(_lib, name) for name in EXPORTED})
