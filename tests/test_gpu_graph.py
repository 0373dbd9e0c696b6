"""hipGraph capture and replay of batched library calls.

A batch of maps of uneven band-limit, spin and reality is prepared, captured
once (batched inverse followed by batched forward, FP64 and FP32C) and
replayed several times with new inputs copied into the captured buffers; eager
library calls of other shapes (which grow the workspace) and synchronisations
run between the replays.  Every replay must equal the eager result bit for
bit: the graph replays the same kernels with the same arguments.
"""
import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mw(tc):
    import paper_1110_6298_amd as m
    m.library()
    return m


SPECS = [(48, 2, 0), (48, 2, 0), (32, 0, 1), (32, 0, 1), (32, 0, 0), (40, -1, 0), (48, 2, 0)]


def inputs(seed):
    out = []
    for i, (L, s, r) in enumerate(SPECS):
        f = mwsynth.flm_gaussian(L, s, seed=seed + i)
        if r:
            f = mwsynth.make_real_symmetric(f, L)
        out.append(f)
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager(tc, mw, precision):
    print("graph replay precision=%d" % precision, flush=True)
    Ls = [a for a, _, _ in SPECS]
    ss = [b for _, b, _ in SPECS]
    rs = [c for _, _, c in SPECS]
    mw.prepare(Ls, ss, rs, precision=precision)
    flm = [tc.from_numpy(f).cuda() for f in inputs(20000)]
    grids = [tc.empty((L, 2 * L - 1), dtype=tc.float64 if r else tc.complex128, device="cuda")
             for L, _, r in SPECS]
    back = [tc.empty(L * L, dtype=tc.complex128, device="cuda") for L, _, _ in SPECS]

    def step():
        mw.inverse_batch(flm, Ls, ss, rs, precision=precision, outs=grids)
        mw.forward_batch(grids, Ls, ss, rs, precision=precision, outs=back)

    side = tc.cuda.Stream()
    side.wait_stream(tc.cuda.current_stream())
    with tc.cuda.stream(side):
        step()
    tc.cuda.current_stream().wait_stream(side)
    tc.cuda.synchronize()
    graph = tc.cuda.CUDAGraph()
    with tc.cuda.graph(graph):
        step()
    tc.cuda.synchronize()

    for rep in range(4):
        new = inputs(21000 + 100 * rep)
        for t, f in zip(flm, new):
            t.copy_(tc.from_numpy(f))
        graph.replay()
        tc.cuda.synchronize()
        got_grid = [g.cpu().numpy().copy() for g in grids]
        got_back = [b.cpu().numpy().copy() for b in back]
        # eager work of another shape between replays (grows the workspace)
        big = 64 + 16 * rep
        x = mw.inverse(tc.from_numpy(mwsynth.flm_gaussian(big, 1, seed=rep)).cuda(), big, 1, precision=precision)
        mw.forward(x, big, 1, precision=precision)
        tc.cuda.synchronize()
        # the eager result for the same inputs
        step()
        tc.cuda.synchronize()
        for i in range(len(SPECS)):
            assert np.array_equal(got_grid[i], grids[i].cpu().numpy()), (rep, i)
            assert np.array_equal(got_back[i], back[i].cpu().numpy()), (rep, i)
            tol = 1e-12 if precision == 0 else 2e-6
            err = np.abs(got_back[i] - new[i]).max() / np.abs(new[i]).max()
            assert err < tol, (rep, i, err)


def test_capture_without_prepare_fails_cleanly(tc, mw):
    """A call under capture that would need a new plan is rejected before any
    launch (MW_ENOMEM), and capture can end normally."""
    L = 77
    flm = tc.zeros(L * L, dtype=tc.complex128, device="cuda")
    out = tc.empty((L, 2 * L - 1), dtype=tc.complex128, device="cuda")
    graph = tc.cuda.CUDAGraph()
    raised = None
    with tc.cuda.graph(graph):
        try:
            mw.inverse(flm, L, 0, out=out)
        except mw.MWError as e:
            raised = e
    assert raised is not None and raised.status == -2
