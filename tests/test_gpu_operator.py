"""GPU parity: Z4 noise (bit-exact) and the operator in every storage
precision against the FP64 CPU oracle, through the C ABI."""

import numpy as np
import pytest

from lattice_inputs import make_gauge, random_spinor

pytestmark = pytest.mark.gpu

# (dims, kappa, a*mu, eps): tiny, anisotropic ragged (384 sites = 1.5 blocks),
# config-0 lattice, several tiles
LATTICES = [
    ((2, 2, 2, 2), 0.16, 0.03125, 0.3),
    ((2, 4, 6, 8), 0.1632, 0.004, 0.3),
    ((4, 4, 4, 4), 0.160, 0.03125, 0.3),
    ((6, 4, 8, 10), 0.1632, 0.003, 0.25),
]
TOL = {0: 1e-12, 1: 1e-6, 2: 5e-3, 3: 5e-3}


def _ctx(dims, kappa, mu, U, t_bc=-1):
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create(dims, kappa, mu, t_bc)
    tq.tm_gauge_load(ctx, U)
    return ctx


def _to_device(psi, prec):
    import torch
    import paper_1211_0126_amd as tq
    t = torch.from_numpy(np.ascontiguousarray(psi)).cuda()
    if prec == tq.PREC_F64:
        return t
    if prec == tq.PREC_F32:
        return t.to(torch.complex64)
    pair = torch.view_as_real(t).to(torch.float32)
    return pair.to(torch.float16 if prec == tq.PREC_F16 else torch.bfloat16).contiguous()


def _to_host(t, prec):
    import torch
    import paper_1211_0126_amd as tq
    if prec in (tq.PREC_F16, tq.PREC_BF16):
        t = torch.view_as_complex(t.to(torch.float32).contiguous())
    return t.to(torch.complex128).cpu().numpy()


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("dims", [l[0] for l in LATTICES])
def test_noise_bit_exact(orc, dims):
    import paper_1211_0126_amd as tq
    U = make_gauge(dims, 0.3, 1)
    ctx = _ctx(dims, 0.16, 0.01, U)
    ids = [0, 1, 7, 1000, 2**40 + 3]
    eta = tq.tm_noise_z4(ctx, 2000, ids).cpu().numpy()
    for k, j in enumerate(ids):
        assert np.array_equal(eta[k], orc.noise_z4(dims, 2000, j)), (dims, j)
    ctx.close()


@pytest.mark.parametrize("lat", LATTICES)
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_dslash_parity(orc, lat, prec, op):
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = lat
    U = make_gauge(dims, eps, 11)
    ctx = _ctx(dims, kappa, mu, U)
    nrhs = 3
    psi = random_spinor(dims, 5, nrhs)
    x = _to_device(psi, prec)
    out = _to_host(tq.tm_dslash(ctx, op, prec, x), prec)
    xin = _to_host(x, prec)  # the input as stored (rounded for F16/BF16)
    for r in range(nrhs):
        ref = orc.apply_op(dims, -1, kappa, mu, op, U, xin[r])
        assert _rel(out[r], ref) < TOL[prec], (dims, prec, op, r, _rel(out[r], ref))
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_dslash_multi_rhs_paths_agree(orc, prec):
    """n = 1, 2, 4, 8 right-hand sides per launch (1, 2 and 4 per lane) give
    the same result for each right-hand side."""
    import paper_1211_0126_amd as tq
    dims = (4, 4, 6, 8)
    U = make_gauge(dims, 0.25, 3)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    psi = random_spinor(dims, 9, 8)
    x8 = _to_device(psi, prec)
    ref = _to_host(tq.tm_dslash(ctx, tq.OP_M, prec, x8), prec)
    for n in (1, 2, 4):
        for r0 in range(0, 8, n):
            out = _to_host(tq.tm_dslash(ctx, tq.OP_M, prec, x8[r0:r0 + n].contiguous()), prec)
            assert _rel(out, ref[r0:r0 + n]) < 1e-6
    ctx.close()


def test_native_layout_round_trip(orc):
    import torch
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 8)
    U = make_gauge(dims, 0.25, 4)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    for prec in (0, 1, 2, 3):
        psi = random_spinor(dims, 12, 4)
        x = _to_device(psi, prec)
        nb = tq.tm_field_bytes(ctx, prec, 4, tq.LAYOUT_NATIVE)
        nat = torch.empty(nb, dtype=torch.uint8, device="cuda")
        nout = torch.empty(nb, dtype=torch.uint8, device="cuda")
        tq.tm_field_convert(ctx, prec, 4, True, x, nat)
        back = torch.empty_like(x)
        tq.tm_field_convert(ctx, prec, 4, False, nat, back)
        assert torch.equal(back.view(torch.uint8), x.view(torch.uint8))  # bit-exact
        tq.tm_dslash(ctx, tq.OP_M, prec, nat, nout, layout=tq.LAYOUT_NATIVE, nrhs=4)
        out = torch.empty_like(x)
        tq.tm_field_convert(ctx, prec, 4, False, nout, out)
        ref = tq.tm_dslash(ctx, tq.OP_M, prec, x)
        assert torch.equal(out.view(torch.uint8), ref.view(torch.uint8))
    ctx.close()


def test_hop_integer_field_exact(orc):
    """Unit links, small-integer field: H is exact in FP64 and FP32, so the
    indexing is checked bit for bit."""
    import paper_1211_0126_amd as tq
    from lattice_inputs import unit_gauge
    dims = (2, 4, 6, 8)
    U = unit_gauge(dims)
    ctx = _ctx(dims, 0.125, 0.0, U)
    rng = np.random.default_rng(3)
    psi = (rng.integers(-8, 8, (1, 384, 4, 3)) + 1j * rng.integers(-8, 8, (1, 384, 4, 3))).astype(np.complex128)
    ref = orc.apply_op(dims, -1, 0.125, 0.0, orc.OP_HOP, U, psi[0])
    for prec in (0, 1):
        out = _to_host(tq.tm_dslash(ctx, tq.OP_HOP, prec, _to_device(psi, prec)), prec)
        assert np.array_equal(out[0], ref)
    ctx.close()


def test_periodic_time_boundary(orc):
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 4)
    U = make_gauge(dims, 0.3, 8)
    ctx = _ctx(dims, 0.16, 0.03125, U, t_bc=1)
    psi = random_spinor(dims, 2, 1)
    out = _to_host(tq.tm_dslash(ctx, tq.OP_M, 0, _to_device(psi, 0)), 0)
    ref = orc.apply_op(dims, 1, 0.16, 0.03125, orc.OP_M, U, psi[0])
    assert _rel(out[0], ref) < 1e-13
    ctx.close()


def test_invalid_arguments():
    import paper_1211_0126_amd as tq
    with pytest.raises(tq.TmError):
        tq.tm_create((1, 4, 4, 4), 0.16, 0.01)
    with pytest.raises(tq.TmError):
        tq.tm_create((4, 4, 4, 4), 0.16, 0.01, t_bc=0)
    ctx = tq.tm_create((4, 4, 4, 4), 0.16, 0.01)
    import torch
    x = torch.zeros((1, 256, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(tq.TmError) as e:
        tq.tm_dslash(ctx, tq.OP_M, 0, x)  # no gauge loaded
    assert e.value.code == -4
    ctx.close()
