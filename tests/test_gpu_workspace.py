"""The caller-owned device workspace and the output layouts of tsm_solve_batch,
through the C ABI.

tm_create takes the workspace (a torch tensor here); every device buffer of
the context is carved from it, a call whose buffers do not fit returns
TM_ENOMEM before it enqueues work, and no device memory is allocated after
tm_create.  tm_workspace_bytes(caps) is enough for the calls caps describes.
"""

import ctypes

import numpy as np
import pytest
import torch

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27

pytestmark = pytest.mark.gpu

KAPPA, MU = 0.1632, 0.004


def _gauge(dims, seed):
    return make_gauge(dims, 0.25, seed)


def _eo_pair(tq, lp_block=8, hp_block=8):
    lp = tq.solve_params(prec=tq.PREC_F16, tol=1e-2, max_iter=-1, rhs_block=lp_block, true_resid=1,
                         solver=tq.SOLVER_CG_EO)
    hp = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=0.1, rhs_block=hp_block,
                         stop=tq.STOP_TRUE, solver=tq.SOLVER_CG_EO)
    return lp, hp


def test_exact_workspace_runs_tsm_and_matches_a_larger_one():
    """A workspace of exactly tm_workspace_bytes(caps) runs the TSM step caps
    describes; the loops are bitwise those of a context with the library's
    default (larger) workspace, the usage report fits the workspace, and two
    calls in a row give the same loops."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = _gauge(dims, 41)
    mom = momenta_27()
    lp, hp = _eo_pair(tq)
    caps = tq.caps([lp, hp], max_sources=24, max_mom=27, mom_distinct=3)
    need = tq.tm_workspace_bytes(dims, KAPPA, MU, -1, caps)
    print("8^4 exact workspace %d bytes" % need, flush=True)
    ctx = tq.tm_create(dims, KAPPA, MU, -1, caps=caps)
    assert ctx.workspace.numel() == need
    tq.tm_gauge_load(ctx, U)
    a = tq.tsm_loops(ctx, 7, 2, 16, lp, hp, mom, per_source=True)
    b = tq.tsm_loops(ctx, 7, 2, 16, lp, hp, mom, per_source=True)
    use = ctx.workspace_usage()
    ctx.close()
    print("usage %s" % use, flush=True)
    assert use["total"] == need // 256 * 256
    assert use["persistent"] + use["peak_scratch"] <= use["total"]
    assert use["peak_scratch"] > 0
    big = tq.tm_create(dims, KAPPA, MU, -1)
    assert big.workspace.numel() > need
    tq.tm_gauge_load(big, U)
    c = tq.tsm_loops(big, 7, 2, 16, lp, hp, mom, per_source=True)
    big.close()
    for r in (b, c):
        assert np.array_equal(a["loops"], r["loops"])
        assert np.array_equal(a["per_source"], r["per_source"])


def test_undersized_workspace_returns_enomem_and_stays_usable():
    """With room for the links but not for a block of sixteen FP64 sources,
    tsm_solve_batch returns TM_ENOMEM (no sticky error); a single-source
    solve that fits then runs and equals that of a large workspace."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = _gauge(dims, 42)
    ref_ctx = tq.tm_create(dims, KAPPA, MU, -1)
    tq.tm_gauge_load(ref_ctx, U)
    persistent = ref_ctx.workspace_usage()["persistent"]
    p1 = tq.solve_params(prec=tq.PREC_F32, tol=1e-6, max_iter=-1, rhs_block=1)
    ref, _, _ = tq.tsm_solve_batch(ref_ctx, p1, 3, [5])
    ref = ref.cpu()
    ref_ctx.close()
    small = tq.tm_create(dims, KAPPA, MU, -1, workspace_bytes=persistent + (8 << 20))
    tq.tm_gauge_load(small, U)
    big_p = tq.solve_params(prec=tq.PREC_F64, tol=1e-6, max_iter=-1, rhs_block=16)
    print("8^4 FP64 block of 16 in a workspace of %d bytes" % small.workspace.numel(), flush=True)
    with pytest.raises(tq.TmError) as ei:
        tq.tsm_solve_batch(small, big_p, 3, list(range(16)))
    assert ei.value.code == tq.binding.TM_ENOMEM
    assert "workspace too small" in str(ei.value)
    got, st, _ = tq.tsm_solve_batch(small, p1, 3, [5])
    assert st[0]["converged"]
    assert torch.equal(got.cpu(), ref)
    small.close()


def test_no_device_allocation_after_create():
    """Free device memory is the same before and after two TSM steps whose
    scratch is several hundred MB: every buffer comes from the workspace."""
    import paper_1211_0126_amd as tq
    dims = (16, 16, 16, 16)
    U = _gauge(dims, 43)
    mom = momenta_27()
    lp, hp = _eo_pair(tq, 16, 8)
    caps = tq.caps([lp, hp], max_sources=40, max_mom=27, mom_distinct=3)
    ctx = tq.tm_create(dims, KAPPA, MU, -1, caps=caps)
    tq.tm_gauge_load(ctx, U)
    # a first step outside the window: graph objects and code objects the
    # runtime loads on first use
    tq.tsm_loops(ctx, 9, 2, 32, lp, hp, mom)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(2):
        tq.tsm_loops(ctx, 9, 2, 32, lp, hp, mom)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    use = ctx.workspace_usage()
    ctx.close()
    print("16^4: free before %d after %d, peak scratch %d" % (free0, free1, use["peak_scratch"]), flush=True)
    assert use["peak_scratch"] > (256 << 20)
    assert abs(free0 - free1) < (16 << 20)


def test_library_allocated_workspace():
    """A null dev_ws makes tm_create allocate ws_bytes once (released by
    tm_destroy); the solves equal those of a torch workspace."""
    import paper_1211_0126_amd as tq
    from paper_1211_0126_amd import binding as B
    dims = (4, 4, 4, 8)
    U = _gauge(dims, 44)
    p = tq.solve_params(prec=tq.PREC_F32, tol=1e-8, max_iter=-1, rhs_block=4, solver=tq.SOLVER_CG_EO)
    ref_ctx = tq.tm_create(dims, KAPPA, MU, -1)
    tq.tm_gauge_load(ref_ctx, U)
    ref, _, _ = tq.tsm_solve_batch(ref_ctx, p, 5, list(range(4)))
    nbytes = ref_ctx.workspace.numel()
    ref_ctx.close()
    lib = B.load_library()
    lat = B._lattice(dims, KAPPA, MU, -1)
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream()
    assert lib.tm_create(ctypes.byref(lat), None, nbytes, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)) == 0
    ctx = B.Context.__new__(B.Context)
    ctx.lib, ctx.h, ctx.dims, ctx.V, ctx.workspace, ctx.stream = lib, h, dims, int(np.prod(dims)), None, stream
    ctx.kappa, ctx.mu, ctx.t_bc = KAPPA, MU, -1
    tq.tm_gauge_load(ctx, U)
    got, _, _ = tq.tsm_solve_batch(ctx, p, 5, list(range(4)))
    assert ctx.workspace_usage()["total"] == nbytes // 256 * 256
    ctx.close()
    assert torch.equal(got, ref)


@pytest.mark.parametrize("reliable", [0, 1])
def test_out_layout_and_precision(reliable):
    """tsm_solve_batch writes the solutions canonical or native, in FP64,
    FP32, FP16 or BF16: each is the FP64 canonical output rounded to nearest
    (bitwise), and the native outputs convert to the canonical ones."""
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 8)
    U = _gauge(dims, 45)
    ctx = tq.tm_create(dims, KAPPA, MU, -1)
    tq.tm_gauge_load(ctx, U)
    ids = [2, 3, 5]
    base = dict(prec=tq.PREC_F32, tol=1e-8, max_iter=-1, rhs_block=2, reliable=reliable, delta=0.1,
                solver=tq.SOLVER_CG_EO)
    out = {}
    for layout in (tq.LAYOUT_CANONICAL, tq.LAYOUT_NATIVE):
        for prec in (tq.PREC_F64, tq.PREC_F32, tq.PREC_F16, tq.PREC_BF16):
            p = tq.solve_params(out_layout=layout, out_prec=prec, **base)
            print("out layout %d prec %d reliable %d" % (layout, prec, reliable), flush=True)
            out[layout, prec], _, _ = tq.tsm_solve_batch(ctx, p, 11, ids)
    s64 = out[tq.LAYOUT_CANONICAL, tq.PREC_F64]
    assert s64.dtype == torch.complex128 and tuple(s64.shape) == (3, ctx.V, 4, 3)
    assert torch.equal(out[tq.LAYOUT_CANONICAL, tq.PREC_F32], s64.to(torch.complex64))
    r32 = torch.view_as_real(s64.to(torch.complex64))
    for prec, dt in ((tq.PREC_F16, torch.float16), (tq.PREC_BF16, torch.bfloat16)):
        got = out[tq.LAYOUT_CANONICAL, prec]
        assert got.dtype == dt and tuple(got.shape) == (3, ctx.V, 4, 3, 2)
        assert torch.equal(got, r32.to(dt))
    for prec in (tq.PREC_F64, tq.PREC_F32, tq.PREC_F16, tq.PREC_BF16):
        nat = out[tq.LAYOUT_NATIVE, prec]
        assert nat.numel() == tq.tm_field_bytes(ctx, prec, 3, tq.LAYOUT_NATIVE)
        canon = torch.empty_like(out[tq.LAYOUT_CANONICAL, prec])
        tq.tm_field_convert(ctx, prec, 3, False, nat, canon)
        torch.cuda.synchronize()
        assert torch.equal(canon, out[tq.LAYOUT_CANONICAL, prec]), prec
    with pytest.raises(tq.TmError):
        tq.tsm_solve_batch(ctx, tq.solve_params(out_layout=5, **base), 11, ids)
    ctx.close()
