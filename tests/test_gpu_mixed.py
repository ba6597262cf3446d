"""Reduced-precision sigma (FP32 / BF16 matrix cores, FP32 accumulation) and the
mixed-precision solve with FP64 residual correction, against the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ssfno
from oracle.adc_cs import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_05897_amd as adc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec,tol", [(1, 2e-5), (2, 3e-2)])
@pytest.mark.parametrize("level", [2, 3])
def test_reduced_precision_sigma_error(prec, tol, level):
    eo, ev, B = synth.make_instance(4, 24, 50, 9, scale=0.5)
    P = Problem(eo, ev, B)
    ctx = adc.Context(dev(eo), dev(ev), dev(B), level, precision=prec)
    r = np.random.default_rng(5).standard_normal((3, P.dim()))
    ref = P.sigma(r, level)
    s64 = host(ctx.sigma(dev(r), precision=0))
    slo = host(ctx.sigma(dev(r), precision=prec))
    assert np.abs(s64 - ref).max() < 1e-11 * np.abs(ref).max()
    err = np.abs(slo - ref).max() / np.abs(ref).max()
    assert 0 < err < tol, err
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_solve_matches_fp64_oracle(prec):
    """Roots of the mixed-precision solve agree with the FP64 oracle within 1e-6 Eh."""
    o, v, X, seed, sc = 3, 10, 24, 8, 0.3
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=sc)
    ref = ssfno.run(eo, ev, B, 3, 1e-4, 1e-2, 1e-9)
    opts = adc.adc3_default_opts()
    opts.precision = prec
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 1e-4, 1e-2, 1e-8, opts)
    assert st == adc.ADC3_OK
    err = np.abs(roots - ref["roots"])
    print("precision", prec, "root errors vs FP64 oracle", err)
    assert err.max() < 1e-6
    assert [r["nvir_kept"] for r in reps] == list(ref["nvir_kept"])


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_solve_weak_correlation_full_size(prec):
    """Workload o=20, v=200, X=600, seed 1, B x 0.018: mixed roots vs stored FP64 oracle roots."""
    gold = json.load(open(os.path.join(HERE, "golden", "ssfno-o20v200x600_s0.018.json")))
    p, eo, ev, B = synth.preset("ssfno-o20v200x600", scale=0.018)
    opts = adc.adc3_default_opts()
    opts.precision = prec
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 5, p["fno_thresh"], p["naf_thresh"], 1e-6, opts)
    assert st == adc.ADC3_OK
    err = np.abs(roots - np.array(gold["roots"]))
    print("precision", prec, "root errors vs FP64 oracle", err)
    assert err.max() < 1e-6
    assert [r["nvir_kept"] for r in reps] == gold["nvir_kept"]
    assert [r["naux_kept"] for r in reps] == gold["naux_kept"]


# FP32 ladder from three 16-row blocks on (33 rows, n_vec * o): the kernel with the packed rows k-major in FP32, both tiles
# copied into LDS by buffer loads.  One and two row tiles, ragged column tiles, 1, 3 or tuned K chunks;
# the FP32 sigma error against the FP64 oracle stays at the FP32 level of the small case above.
@pytest.mark.parametrize("o,v,X,nvec", [(6, 41, 60, 7), (10, 41, 60, 16), (8, 80, 120, 9), (16, 45, 70, 4),
                                        (16, 45, 70, 6), (20, 44, 66, 5), (16, 45, 70, 8)], ids=lambda c: str(c))
@pytest.mark.parametrize("chunks", ["", "1", "3"])
def test_fp32_sigma_stored_ladder_row_tiles(o, v, X, nvec, chunks, monkeypatch):
    monkeypatch.setenv("ADC3_LADDER_CHUNKS", chunks)
    eo, ev, B = synth.make_instance(o, v, X, 7, scale=0.3)
    P = Problem(eo, ev, B)
    ctx = adc.Context(dev(eo), dev(ev), dev(B), 3, nroots=0, precision=1)
    r = np.random.default_rng(3).standard_normal((nvec, P.dim()))
    ref = P.sigma(r, 3)
    slo = host(ctx.sigma(dev(r), precision=1))
    ctx.close()
    err = np.abs(slo - ref).max() / np.abs(ref).max()
    assert 0 < err < 2e-5, err
