"""The ladder entry point that allocates nothing (adc3_ladder_apply_static, scratch in a static device
array) against the workspace entry point (adc3_ladder_apply) and the FP64 oracle: two calls in a row,
the second with a smaller input, in FP64, FP32 and BF16 operands; a shape beyond the static scratch is
rejected before any launch.

With the workspace entry point given exactly the static array's size, both split the auxiliary
functions into the same chunks and run the same kernels, so their results agree bit for bit."""
import numpy as np
import pytest

import synth
from oracle.adc_cs import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_05897_amd as adc  # noqa: E402

TOL = {0: 1e-12, 1: 2e-5, 2: 3e-2}


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_static_ladder_matches_workspace_ladder(prec):
    cases = [(48, 150, 40, 3), (20, 33, 7, 4)]  # (v, X, rows, seed); the second call is smaller
    for v, X, M, seed in cases:
        print("static ladder v=%d X=%d rows=%d precision %d" % (v, X, M, prec), flush=True)
        eo, ev, B = synth.make_instance(2, v, X, seed, scale=0.5)
        P = Problem(eo, ev, B)
        Z = np.random.default_rng(seed).standard_normal((M, v, v))
        Bd, Zd = dev(P.Bvv), dev(Z)
        out = torch.full_like(Zd, float("nan"))
        before = torch.cuda.memory_allocated()
        adc.adc3_ladder_apply_static(Bd, Zd, precision=prec, out=out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = host(out)
        ref_ws = host(adc.adc3_ladder_apply(Bd, Zd, precision=prec, workspace_bytes=adc.STATIC_SCRATCH_BYTES))
        assert np.array_equal(got, ref_ws)
        ref = P.vvvv_apply(Z)
        assert np.abs(got - ref).max() < TOL[prec] * np.abs(ref).max()


def test_static_ladder_rejects_shapes_beyond_the_scratch():
    v, X, M = 400, 300, 220  # intermediate of one auxiliary function alone: 220 * 400^2 * 8 B = 282 MB
    assert adc.adc3_ladder_workspace_bytes(v, X, M, 0) > adc.STATIC_SCRATCH_BYTES
    Bd = torch.zeros((X, v, v), dtype=torch.float64, device="cuda")
    Zd = torch.zeros((M, v, v), dtype=torch.float64, device="cuda")
    with pytest.raises(adc.ADCError) as e:
        adc.adc3_ladder_apply_static(Bd, Zd)
    assert e.value.status == adc.ADC3_ENOMEM
    assert "static scratch" in str(e.value)
