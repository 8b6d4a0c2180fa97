import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# tests run the built-in tile rules, not the tuning file beside the library
# (tuned values change speed only; tests that read a tuning file set their own)
os.environ.setdefault("PHG_TUNE", "off")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "fp32_routed: an FP32 context of this test may be evaluated in FP64 "
                                       "by the precision guard")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(autouse=True)
def _fp32_contexts_run_fp32(request, monkeypatch):
    """In GPU tests, an FP32 context's evaluation must run the float32 kernels
    unless the test is marked fp32_routed: a parity result claimed for FP32
    must not silently come from the FP64 twin of the precision guard."""
    if request.node.get_closest_marker("gpu") is None or request.node.get_closest_marker("fp32_routed"):
        yield
        return
    from paper_2303_04390_amd import binding as B
    orig = B.Context.gradient

    def gradient(self):
        out = orig(self)
        if self.prec == B.PHG_FP32_SCALED:
            assert B.phg_last_precision(self.handle) == B.PHG_FP32_SCALED, \
                "the FP32 precision guard routed this evaluation to FP64"
        return out

    monkeypatch.setattr(B.Context, "gradient", gradient)
    yield
