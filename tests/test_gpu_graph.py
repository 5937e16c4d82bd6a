"""SpMV of every implementation class captured in a HIP graph (through
torch's CUDA-graph API) and replayed.  A product launches only kernels on
the context's stream (no allocation, no memset, no host synchronisation),
which is what capture needs; every replay must equal the eager product bit
for bit, with eager work and synchronisations between the replays.
"""
import ctypes

import pytest

import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
xab = pytest.importorskip("paper_2405_01599_amd")

CASES = [(False, k) for k in xab.GENERAL_CLASSES] + [(True, k) for k in xab.SYM_CLASSES]


@pytest.fixture(scope="module")
def ctx():
    return xab.Context(0)


@pytest.fixture(scope="module")
def mats(ctx):
    # a band (4 x 4 blocks fill it well enough for the block CSR copy) and
    # the lower triangle of a 27-point stencil
    return {False: ctx.matrix_from_csr(gen.banded(20_000, 8, seed=31)),
            True: ctx.matrix_from_csr(gen.stencil27(24, lower=True))}


def _set_stream(ctx, s):
    assert xab.lib().xab_set_stream(ctx.h, ctypes.c_void_p(s.cuda_stream)) == 0


@pytest.mark.parametrize("lower,k", CASES)
def test_spmv_graph_replay_equals_eager(ctx, mats, lower, k):
    M = mats[lower]
    P = ctx.plan_class(M, k)
    if k == 9:
        # the atomic baseline adds in arrival order: integer x keeps every
        # order exact
        x = torch.from_numpy(gen.int_vec(M.n, 5)).cuda().to(torch.float64)
    else:
        x = torch.from_numpy(gen.uniform_vec(M.n, 5)).cuda()
    main = torch.cuda.current_stream()
    y_eager = ctx.spmv(P, x)
    torch.cuda.synchronize()
    y = torch.empty_like(y_eager)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    try:
        _set_stream(ctx, s)
        s.wait_stream(main)
        with torch.cuda.stream(s):
            ctx.spmv(P, x, y)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            ctx.spmv(P, x, y)
    finally:
        _set_stream(ctx, main)
    torch.cuda.synchronize()
    for _ in range(3):
        y.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager)
        y2 = ctx.spmv(P, x)  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(y2, y_eager)
