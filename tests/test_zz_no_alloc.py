"""vds_pair_sums_noalloc (the entry point for callers that cannot allocate
device memory): through the C ABI on contexts with no workspace bound, its
results equal those of vds_pair_sums on a bound workspace bit for bit (the
same kernels on the same inputs), on two calls in a row that share the static
scratch, the second with a smaller problem; a problem larger than the scratch
is rejected before any launch, and a bound workspace stays bound."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vds():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2603_12550_amd import _vds
    return _vds


def _raw_ctx(vds, nb, P, h, G):
    """A context created through the C ABI with no workspace bound."""
    import torch
    prob = vds.make_problem(nb, P, h, G=G, scheme="explicit")
    H = (C.c_double * nb)(*([1.0] * nb))
    ctx = C.c_void_p()
    st = vds._lib.vds_create(C.byref(prob), H, C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(ctx))
    assert st == vds.VDS_OK
    return ctx


def _noalloc(vds, ctx, q, w, P, nb):
    import torch
    S = torch.empty(P, dtype=torch.float32, device="cuda")
    t1 = torch.empty((nb, P, 3), dtype=torch.float32, device="cuda")
    t2 = torch.empty_like(t1)
    st = vds._lib.vds_pair_sums_noalloc(ctx, vds._ptr(q), vds._ptr(w), vds._ptr(S), vds._ptr(t1), vds._ptr(t2))
    return st, S, t1, t2


def test_noalloc_pair_sums_equal_the_bound_workspace_form(vds):
    import torch
    cases = [(3, 20000, 0.4, wl.shear_gradient(1.0), 2, None),      # the 4-bead chain at full size
             (3, 1500, 0.45, wl.shear_gradient(0.5), 7, 11)]        # then a smaller problem, random weights
    for nb, P, h, G, seed, wseed in cases:
        _say(f"noalloc pair sums nb={nb} P={P}")
        q = torch.from_numpy(wl.to_f32(wl.gaussian_bonds(seed, nb, P, 1 / 3))).cuda()
        w = None if wseed is None else torch.from_numpy(wl.to_f32(wl.random_weights(wseed, P))).cuda()
        ctx = _raw_ctx(vds, nb, P, h, G)
        try:
            st, S, t1, t2 = _noalloc(vds, ctx, q, w, P, nb)
            assert st == vds.VDS_OK, vds._lib.vds_last_error(ctx)
            torch.cuda.synchronize()
            ref = vds.Context(nb, P, h, G=G, scheme="explicit", poison=True)
            S_r, t1_r, t2_r = ref.pair_sums(q, w)
            for a, b in ((S, S_r), (t1, t1_r), (t2, t2_r)):
                assert bool(torch.isfinite(a).all().item())
                assert bool((a == b).all().item())
        finally:
            vds._lib.vds_destroy(ctx)


def test_noalloc_rejects_a_problem_larger_than_the_scratch_and_keeps_a_bound_workspace(vds):
    import torch
    P = 40000  # the 4-bead chain needs more than the 64 MiB scratch here
    ctx = _raw_ctx(vds, 3, P, 0.4, wl.shear_gradient(1.0))
    try:
        q = torch.zeros((3, P, 3), dtype=torch.float32, device="cuda")
        st, *_ = _noalloc(vds, ctx, q, None, P, 3)
        assert st == vds.VDS_ERR_ARG
        assert b"static scratch" in vds._lib.vds_last_error(ctx)
    finally:
        vds._lib.vds_destroy(ctx)
    # on a context with a bound workspace: the same results, and the workspace
    # is still the context's afterwards
    P, nb, h = 900, 3, 0.5
    c = vds.Context(nb, P, h, G=wl.shear_gradient(1.0), scheme="explicit", poison=True)
    q = torch.from_numpy(wl.to_f32(wl.gaussian_bonds(5, nb, P, 1 / 3))).cuda()
    S0, a0, b0 = c.pair_sums(q)
    st, S1, a1, b1 = _noalloc(vds, c.ctx, q, None, P, nb)
    assert st == vds.VDS_OK
    S2, a2, b2 = c.pair_sums(q)
    for x, y, z in ((S0, S1, S2), (a0, a1, a2), (b0, b1, b2)):
        assert bool((x == y).all().item()) and bool((x == z).all().item())
