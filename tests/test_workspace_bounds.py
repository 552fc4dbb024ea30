"""tm_workspace_bytes (host code only, no GPU): the bound grows with what the
caps ask for, covers at least the links the context keeps, is independent of
the order of the listed solves, and is 0 for lattices or caps the library
refuses."""

import ctypes

import pytest


@pytest.fixture(scope="module")
def tq():
    import os

    import paper_1211_0126_amd as tq
    if not os.path.exists(tq.LIB_PATH):
        from paper_1211_0126_amd.build import build
        build()
    tq.load_library()
    return tq


DIMS = (8, 8, 8, 16)


def _b(tq, caps, dims=DIMS):
    return tq.tm_workspace_bytes(dims, 0.16, 0.01, -1, caps)


def _lp(tq, block=16, prec=2, solver=2, **kw):
    return tq.solve_params(prec=prec, rhs_block=block, solver=solver, **kw)


def test_links_are_a_lower_bound(tq):
    # FP64 (576 B) + FP32 (192 B) + bfloat16 (192 B) links per site, and the
    # parity-split FP32, FP64 and binary16 copies again: at least 1920 B a site
    v = 8 * 8 * 8 * 16
    assert _b(tq, tq.caps([])) >= 1920 * v


def test_monotone_in_block_sources_momenta_and_estimators(tq):
    base = _b(tq, tq.caps([_lp(tq, 8)], max_sources=16))
    assert _b(tq, tq.caps([_lp(tq, 16)], max_sources=16)) > base
    assert _b(tq, tq.caps([_lp(tq, 8)], max_sources=4096)) > base
    assert _b(tq, tq.caps([_lp(tq, 8)], max_sources=16, max_mom=64, mom_distinct=4)) > base
    assert _b(tq, tq.caps([_lp(tq, 8)], max_sources=16, estimators=(0, 3))) > base
    assert _b(tq, tq.caps([_lp(tq, 8)], max_sources=16, train_pairs=64, train_sources=8)) > base


def test_reliable_and_fp64_solves_need_more_than_fp16(tq):
    f16 = _b(tq, tq.caps([_lp(tq, 16)]))
    rel = _b(tq, tq.caps([_lp(tq, 16, prec=1, reliable=1, stop=1)]))
    f64 = _b(tq, tq.caps([_lp(tq, 16, prec=0, solver=0)]))
    assert rel > f16 and f64 > f16


def test_two_settings_are_summed_for_tsm_loops(tq):
    """tsm_loops holds an LP and an HP block at once: listing a second
    setting adds its block, whatever the order."""
    lp, hp = _lp(tq, 32), _lp(tq, 16, prec=1, reliable=1, stop=1)
    one = _b(tq, tq.caps([lp]))
    both = _b(tq, tq.caps([lp, hp]))
    assert both == _b(tq, tq.caps([hp, lp]))
    assert both > one


def test_null_caps_cover_a_typical_listing(tq):
    lp, hp = _lp(tq, 32), _lp(tq, 16, prec=1, reliable=1, stop=1)
    assert _b(tq, None) >= _b(tq, tq.caps([lp, hp], max_sources=256))


def test_refused_lattices_and_caps_give_zero(tq):
    assert _b(tq, None, dims=(1, 4, 4, 4)) == 0
    assert _b(tq, None, dims=(48, 48, 48, 96)) == 0
    c = tq.caps([])
    c.n_solves = 5
    assert _b(tq, c) == 0
    c = tq.caps([])
    c.max_sources = -1
    assert _b(tq, c) == 0


def test_caps_struct_matches_header(tq):
    # the binding's Caps has the header's field order (the layout test
    # compiles the header); here only the size of the solve array
    assert ctypes.sizeof(tq.Caps) > tq.binding.CAPS_MAX_SOLVES * ctypes.sizeof(tq.binding.SolveParams)
