"""phg_gradient_async_noalloc (workspace in the library's static device array)
against phg_gradient_async (workspace the library allocates) on the same
inputs: bitwise-equal results, for two calls in a row with the second on a
smaller problem, for both precisions and for 4 and 20 states, and again for
the first problem after the second one overwrote the shared array."""
import numpy as np
import pytest

from paper_2303_04390_amd import binding as B
from paper_2303_04390_amd import synth

pytestmark = pytest.mark.gpu


def _problems(prec):
    big = (200, 3000) if prec == B.PHG_FP32_SCALED else (200, 1500)
    return [("hky200", synth.config_problem("hky1000", seed=5, n_tips=big[0], n_patterns=big[1])),
            ("hky16", synth.config_problem("hky16", seed=2, n_patterns=500)),
            ("aa60", synth.config_problem("aa500", seed=1, n_tips=60, n_patterns=500))]


def _eval(h, fn, stream, E):
    import torch
    out = torch.full((1 + E,), float("nan"), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        fn(h, out.data_ptr(), out.data_ptr() + 8)
    stream.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [B.PHG_FP32_SCALED, B.PHG_FP64])
def test_noalloc_matches_allocating_entry(prec):
    import torch
    stream = torch.cuda.Stream()
    probs = _problems(prec)
    refs, statics = [], []
    try:
        for name, prob in probs:
            E = 2 * prob.n_tips - 2
            with B.Context.for_problem(prob, prec) as ctx:
                B.phg_bind_stream(ctx.handle, stream.cuda_stream)
                refs.append(_eval(ctx.handle, B.phg_gradient_async, stream, E))
            s = B.Context.for_problem(prob, prec)
            B.phg_bind_stream(s.handle, stream.cuda_stream)
            statics.append(s)
        # first call, then a second one on a smaller problem, then the rest,
        # then the first problem again after the others overwrote the array
        order = [0, 1, 2, 0, 2]
        for i in order:
            name, prob = probs[i]
            print(f"[case] noalloc {name} prec={prec}", flush=True)
            got = _eval(statics[i].handle, B.phg_gradient_async_noalloc, stream, 2 * prob.n_tips - 2)
            assert np.all(np.isfinite(got)), name
            assert np.array_equal(got, refs[i]), (name, np.max(np.abs(got - refs[i])))
    finally:
        for s in statics:
            s.close()


def test_noalloc_refusals():
    import torch
    prob = synth.config_problem("hky16", seed=2, n_patterns=100)
    print("[case] noalloc refusals", flush=True)
    out = torch.zeros(31, dtype=torch.float64, device="cuda")
    # no bound stream
    with B.Context.for_problem(prob, B.PHG_FP32_SCALED) as ctx:
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient_async_noalloc(ctx.handle, out.data_ptr(), out.data_ptr() + 8)
        assert e.value.status == B.PHG_ERR_STATE
        # evaluated in its own memory first: refused afterwards
        ctx.gradient()
        stream = torch.cuda.Stream()
        B.phg_bind_stream(ctx.handle, stream.cuda_stream)
        with pytest.raises(B.PhgError) as e:
            B.phg_gradient_async_noalloc(ctx.handle, out.data_ptr(), out.data_ptr() + 8)
        assert e.value.status == B.PHG_ERR_STATE
