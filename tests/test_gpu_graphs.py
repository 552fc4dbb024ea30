"""Graph-captured CG chunks give the same results as eager launches, on
every replay, with eager work and synchronisations between replays."""

import pytest

from lattice_inputs import make_gauge

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,reliable", [(3, 0), (1, 1), (0, 0)])
def test_graph_replays_match_eager(prec, reliable):
    import torch
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = make_gauge(dims, 0.25, 9)
    stream = torch.cuda.Stream()  # graphs need a non-null stream (default priority)
    with torch.cuda.stream(stream):
        ctx = tq.tm_create(dims, 0.1632, 0.004, -1, stream=stream)
        tq.tm_gauge_load(ctx, U)
        tol = 1e-10 if reliable else 1e-2
        p = tq.solve_params(prec=prec, tol=tol, max_iter=-1, reliable=reliable, rhs_block=4)
        ids = [0, 1, 2, 3]
        tq.tm_set_graphs(ctx, False)
        ref, st_ref, _ = tq.tsm_solve_batch(ctx, p, 5, ids)
        n0 = tq.tm_set_graphs(ctx, True)
        for rep in range(3):
            sol, st, _ = tq.tsm_solve_batch(ctx, p, 5, ids)
            assert torch.equal(sol, ref), rep
            assert [s["iters"] for s in st] == [s["iters"] for s in st_ref]
            # eager work on the stream between replays
            tq.tm_noise_z4(ctx, 7, [rep])
            stream.synchronize()
        assert tq.tm_set_graphs(ctx) > n0
        ctx.close()
