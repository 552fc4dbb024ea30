"""The allocation-free operator entry point (tm_dslash_noalloc) against
tm_dslash through the C ABI: identical kernels, so identical bits, on two
calls in a row (the second with fewer right-hand sides), in both layouts and
every op; a call whose scratch need exceeds the fixed maximum is refused
before anything runs, and the context stays usable."""

import numpy as np
import pytest

from lattice_inputs import make_gauge, random_spinor

pytestmark = pytest.mark.gpu

DIMS, KAPPA, MU = (4, 6, 4, 8), 0.1632, 0.004


def _dev(psi, prec):
    import torch
    import paper_1211_0126_amd as tq
    t = torch.from_numpy(np.ascontiguousarray(psi)).cuda()
    if prec == tq.PREC_F64:
        return t
    if prec == tq.PREC_F32:
        return t.to(torch.complex64)
    pair = torch.view_as_real(t).to(torch.float32)
    return pair.to(torch.float16 if prec == tq.PREC_F16 else torch.bfloat16).contiguous()


@pytest.fixture(scope="module")
def ctx():
    import paper_1211_0126_amd as tq
    U = make_gauge(DIMS, 0.25, 31)
    c = tq.tm_create(DIMS, KAPPA, MU, -1)
    tq.tm_gauge_load(c, U)
    yield c
    c.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_noalloc_canonical_matches_dslash(ctx, prec, op):
    import torch
    import paper_1211_0126_amd as tq
    for k, nrhs in enumerate((4, 2)):  # second call: smaller input
        x = _dev(random_spinor(DIMS, 100 + 10 * op + k, nrhs), prec)
        ref = tq.tm_dslash(ctx, op, prec, x)
        out = torch.full_like(x, float("nan"))
        tq.tm_dslash_noalloc(ctx, op, prec, x, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (prec, op, nrhs)


@pytest.mark.parametrize("op", [0, 2])
def test_noalloc_native_matches_dslash(ctx, op):
    import torch
    import paper_1211_0126_amd as tq
    prec = tq.PREC_F32
    for k, nrhs in enumerate((3, 1)):
        x = _dev(random_spinor(DIMS, 200 + k, nrhs), prec)
        nb = tq.tm_field_bytes(ctx, prec, nrhs, tq.LAYOUT_NATIVE)
        xn = torch.zeros(nb, dtype=torch.uint8, device="cuda")
        tq.tm_field_convert(ctx, prec, nrhs, 1, x, xn)
        ref = torch.zeros_like(xn)
        out = torch.zeros_like(xn)
        tq.tm_dslash(ctx, op, prec, xn, ref, layout=tq.LAYOUT_NATIVE, nrhs=nrhs)
        tq.tm_dslash_noalloc(ctx, op, prec, xn, out, layout=tq.LAYOUT_NATIVE, nrhs=nrhs)
        a = torch.empty_like(x)
        b = torch.empty_like(x)
        tq.tm_field_convert(ctx, prec, nrhs, 0, ref, a)
        tq.tm_field_convert(ctx, prec, nrhs, 0, out, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (op, nrhs)


def test_noalloc_rejects_oversized_call():
    import torch
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    c = tq.tm_create(dims, KAPPA, MU, -1)
    tq.tm_gauge_load(c, make_gauge(dims, 0.25, 5))
    # canonical FP64 M^dag M of 60 right-hand sides needs three native
    # fields of 60 * 835,584 bytes (150 MB) > 128 MiB
    nrhs = 60
    need = 3 * ((tq.tm_field_bytes(c, tq.PREC_F64, nrhs, tq.LAYOUT_NATIVE) + 255) // 256 * 256)
    assert need > 128 << 20
    x = torch.zeros((nrhs, 4096, 4, 3), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(x)
    with pytest.raises(tq.TmError) as ei:
        tq.tm_dslash_noalloc(c, tq.OP_MDAGM, tq.PREC_F64, x, out)
    assert ei.value.code == -1 and "maximum" in str(ei.value)
    # the refusal is not sticky: a call that fits still runs and agrees
    y = _dev(random_spinor(dims, 9, 2), tq.PREC_F64)
    ref = tq.tm_dslash(c, tq.OP_MDAGM, tq.PREC_F64, y)
    got = torch.empty_like(y)
    tq.tm_dslash_noalloc(c, tq.OP_MDAGM, tq.PREC_F64, y, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    c.close()


def test_noalloc_matches_oracle(ctx, orc):
    """The allocation-free path to the operator's FP64 bar (1e-12)."""
    import torch
    import paper_1211_0126_amd as tq
    U = make_gauge(DIMS, 0.25, 31)
    psi = random_spinor(DIMS, 300, 2)
    x = _dev(psi, tq.PREC_F64)
    out = torch.empty_like(x)
    tq.tm_dslash_noalloc(ctx, tq.OP_MDAGM, tq.PREC_F64, x, out)
    got = out.cpu().numpy()
    for r in range(2):
        ref = orc.apply_op(DIMS, -1, KAPPA, MU, 2, U, psi[r])
        assert np.linalg.norm(got[r] - ref) / np.linalg.norm(ref) < 1e-12
