"""One whole evaluation captured as a HIP graph (through torch's graph
capture on the context's bound stream) and replayed: every replay equals the
eager result bit for bit, with eager work and synchronisations between
replays, and replays after new branch lengths are uploaded (phg_prepare)
follow them."""
import numpy as np
import pytest

from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_graph_replay_matches_eager(prec):
    import torch
    prob = synth.config_problem("hky1000", seed=3, n_tips=300, n_patterns=2000)
    E = 2 * prob.n_tips - 2
    print(f"[case] graph replay prec={prec}", flush=True)
    stream = torch.cuda.Stream()
    out = torch.zeros(1 + E, dtype=torch.float64, device="cuda")
    gout = torch.zeros(1 + E, dtype=torch.float64, device="cuda")
    with B.Context.for_problem(prob, prec) as ctx:
        h = ctx.handle
        B.phg_bind_stream(h, stream.cuda_stream)

        def eager():
            with torch.cuda.stream(stream):
                B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)
            torch.cuda.synchronize()
            return out.cpu().numpy().copy()

        ref = eager()                       # also uploads every input
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            B.phg_bind_stream(h, torch.cuda.current_stream().cuda_stream)
            B.phg_gradient_async(h, gout.data_ptr(), gout.data_ptr() + 8)
        B.phg_bind_stream(h, stream.cuda_stream)
        for i in range(4):
            gout.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(gout.cpu().numpy(), ref), i
            assert np.array_equal(eager(), ref)
        # new branch lengths: upload, then the same graph computes with them
        b2 = prob.b * np.exp(np.random.default_rng(1).normal(0.0, 0.05, E))
        B.phg_set_branch_lengths(h, b2)
        B.phg_prepare(h)
        ref2 = eager()
        assert not np.array_equal(ref2, ref)
        for i in range(2):
            gout.zero_()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(gout.cpu().numpy(), ref2), i


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
@pytest.mark.parametrize("which", ["hky1000", "aa500"])
def test_library_graph_replays_match_launches(prec, which):
    """phg_gradient / phg_log_likelihood replay the context's own captured
    graph while only device data changes; every replay equals a graph-free
    context's launches bit for bit, new branch lengths and a new model flow
    into the replay, and a new topology makes the context capture again."""
    kw = dict(n_tips=200, n_patterns=1500) if which == "hky1000" else dict(n_tips=60, n_patterns=300)
    prob = synth.config_problem(which, seed=4, **kw)
    E = 2 * prob.n_tips - 2
    rng = np.random.default_rng(2)
    print(f"[case] library graph {which} prec={prec}", flush=True)
    with B.Context.for_problem(prob, prec) as g, B.Context.for_problem(prob, prec) as e:
        B.phg_set_graphs(e.handle, False)
        for i in range(5):
            b = prob.b * np.exp(rng.normal(0.0, 0.1, E))
            for c in (g, e):
                B.phg_set_branch_lengths(c.handle, b)
            lg, gg = g.gradient()
            le, ge = e.gradient()
            assert lg == le and np.array_equal(gg, ge), i
            assert g.log_likelihood() == e.log_likelihood() == lg
        caps, reps = B.phg_graph_stats(g.handle)
        assert caps == 2 and reps == 8, (caps, reps)      # one gradient graph, one logL graph
        assert B.phg_graph_stats(e.handle) == (0, 0)
        # a new model: device data only, the graph stays
        pi2 = np.roll(prob.pi, 1)
        for c in (g, e):
            B.phg_set_root_frequencies(c.handle, pi2)
        assert g.gradient()[0] == e.gradient()[0]
        assert B.phg_graph_stats(g.handle)[0] == 2
        # a new topology: a new launch sequence, captured again
        parent2 = synth.yule_topology(prob.n_tips, np.random.default_rng(9))
        for c in (g, e):
            B.phg_set_topology(c.handle, parent2)
            B.phg_set_branch_lengths(c.handle, prob.b)
        lg, gg = g.gradient()
        le, ge = e.gradient()
        assert lg == le and np.array_equal(gg, ge)
        assert B.phg_graph_stats(g.handle)[0] == 3
