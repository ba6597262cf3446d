"""The lockstep block Davidson (opts.lockstep = 1): fixed-shape iterations with the convergence flags on
the device, each solve's chunks of iterations replayed from HIP graphs on its own stream, the block
shrinking to the roots still active at each chunk boundary.  Against the FP64 oracle
(1e-8 Eh FP64, 1e-6 Eh mixed precision) and the one-solve-at-a-time path:

* one canonical solve (tiny dense workload: full diagonalisation of the oracle's matrix);
* the per-root SS-FNO bases of one instance together (truncated ADC(2) solves, then ADC(3)), FP64 and
  FP32 / BF16 ladders, state-specific and shared MP2-FNO bases;
* ragged batches in waves (canonical and truncating instances, FP64 and FP32 ladder with graphs);
* chunk lengths 1 and 4 (ADC3_DAV_CHUNK is read once per process, so the chunk is the default 3 here and
  the graph cache is exercised by the repeating collapse cycle), caller guesses, max_iter, NaN injection.
"""
import numpy as np
import pytest

import synth
from oracle import ssfno
from oracle.adc_cs import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_05897_amd as adc  # noqa: E402


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _opts(**kw):
    o = adc.adc3_default_opts()
    o.lockstep = 1
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_lockstep_canonical_matches_dense_oracle():
    p, eo, ev, B = synth.preset("tiny-dense")
    P = Problem(eo, ev, B)
    ref = np.linalg.eigvalsh(P.dense(3))[:3]
    print("lockstep canonical tiny-dense", flush=True)
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=_opts())
    assert st == adc.ADC3_OK and np.abs(roots - ref).max() < 1e-8
    assert all(r["resnorm"] <= 1e-8 for r in reps)
    for level, x in ((2, 1.0), (3, 0.5)):
        o = _opts(level=level, sm_x=x)
        roots, _, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=o)
        ref = np.linalg.eigvalsh(P.dense(2) if level == 2 else P.dense_sm(x))[:3]
        assert st == adc.ADC3_OK and np.abs(roots - ref).max() < 1e-8, level


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6), (2, 1e-6)])
@pytest.mark.parametrize("mode", [0, 1])
def test_lockstep_per_root_bases_match_oracle(prec, tol, mode):
    eo, ev, B = synth.make_instance(3, 10, 24, 8, scale=0.3)
    refp = ssfno.run(eo, ev, B, 3, 1e-4, 1e-2, 1e-10, fno_mode="mp2" if mode else "ss")
    print("lockstep bases precision %d mode %d" % (prec, mode), flush=True)
    o = _opts(precision=prec, fno_mode=mode)
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 1e-4, 1e-2, 1e-9, opts=o)
    assert st == adc.ADC3_OK
    assert [r["nvir_kept"] for r in reps] == list(refp["nvir_kept"])
    assert [r["naux_kept"] for r in reps] == list(refp["naux_kept"])
    assert np.abs(roots - refp["roots"]).max() < tol
    seq, _, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 1e-4, 1e-2, 1e-9,
                                   opts=_opts(precision=prec, fno_mode=mode, lockstep=0))
    assert np.abs(roots - seq).max() < tol
    if prec == 0:
        assert np.abs(np.array([r["pole_strength"] for r in reps]) - refp["pole_strength"]).max() < 1e-6


def test_lockstep_literal_workload_matches_golden():
    """The benchmark's workload (o=20, v=200, X=600, literal scale) with its five bases in lockstep."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "ssfno-o20v200x600.json")))
    p, eo, ev, B = synth.preset("ssfno-o20v200x600")
    print("lockstep literal o20v200x600", flush=True)
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 5, p["fno_thresh"], p["naf_thresh"], p["conv"],
                                        opts=_opts())
    assert st == adc.ADC3_OK
    assert [r["naux_kept"] for r in reps] == gold["naux_kept"]
    # the bar of the one-at-a-time parity test (FP64 rounding at |omega| = 2.7e6)
    tol = np.maximum(1e-8, 2e-13 * np.abs(np.array(gold["roots"])))
    assert np.all(np.abs(roots - np.array(gold["roots"])) <= tol)


def _ragged(n, seed0, scale):
    out = []
    for s in range(seed0, seed0 + n):
        rng = np.random.default_rng(s)
        o, v = int(rng.integers(2, 6)), int(rng.integers(8, 25))
        out.append(synth.make_instance(o, v, 3 * v, s, scale=scale))
    return out


@pytest.mark.parametrize("prec,graphs", [(0, 0), (1, 1)])
def test_lockstep_ragged_batch_matches_oracle(prec, graphs):
    raw = _ragged(7, 100, 0.3)
    inst = [dict(eps_occ=dev(eo), eps_vir=dev(ev), B=dev(B), nroots=3, conv=1e-8) for eo, ev, B in raw]
    print("lockstep ragged batch precision %d" % prec, flush=True)
    o = _opts(precision=prec, sigma_graphs=graphs)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        roots, reps, sts, st = adc.adc3_ea_solve_batched(inst, opts=o, nstreams=3)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in sts)
    for (eo, ev, B), r in zip(raw, roots):
        ref = np.linalg.eigvalsh(Problem(eo, ev, B).dense(3))[:3]
        assert np.abs(r - ref).max() < (1e-8 if prec == 0 else 1e-6)


def test_lockstep_batch_with_truncating_instances():
    raw = _ragged(4, 120, 0.05)
    inst = [dict(eps_occ=dev(eo), eps_vir=dev(ev), B=dev(B), nroots=2, conv=1e-8, fno_thresh=1e-4,
                 naf_thresh=1e-3) for eo, ev, B in raw]
    inst.append(dict(eps_occ=dev(raw[0][0]), eps_vir=dev(raw[0][1]), B=dev(raw[0][2]), nroots=2, conv=1e-8))
    print("lockstep batch with truncation", flush=True)
    roots, reps, sts, st = adc.adc3_ea_solve_batched(inst, opts=_opts(), nstreams=2)
    assert st == 0
    for (eo, ev, B), r in zip(raw, roots[:4]):
        ref = ssfno.run(eo, ev, B, 2, 1e-4, 1e-3, 1e-10)["roots"]
        assert np.abs(r - ref).max() < 1e-8
    eo, ev, B = raw[0]
    assert np.abs(roots[4] - np.linalg.eigvalsh(Problem(eo, ev, B).dense(3))[:2]).max() < 1e-8


def test_lockstep_guesses_max_iter_and_nan():
    p, eo, ev, B = synth.preset("tiny-dense")
    ref = np.linalg.eigvalsh(Problem(eo, ev, B).dense(3))[:3]
    N = 20 + 4 * 20 * 20
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=_opts(max_iter=1))
    assert st == adc.ADC3_WNOCONV
    vec = torch.zeros((3, N), dtype=torch.float64, device="cuda")
    _, r6, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8,
                                  opts=_opts(max_iter=7, vectors_out=vec.data_ptr()))
    assert st == adc.ADC3_WNOCONV
    fresh, frep, _ = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=_opts())
    res, rrep, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8,
                                      opts=_opts(init_guess=vec.data_ptr(), n_guess=3))
    assert st == adc.ADC3_OK and np.abs(res - ref).max() < 1e-8
    assert rrep[0]["iters"] < frep[0]["iters"]
    adc.adc3_debug_inject_nan(2)
    try:
        with pytest.raises(adc.ADCError) as e:
            adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=_opts())
        assert e.value.status == adc.ADC3_ENUMERIC
    finally:
        adc.adc3_debug_inject_nan(0)


def _golden(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + ".json")))


@pytest.mark.parametrize("prec,conv,tol", [(0, 1e-8, 1e-8), (1, 1e-7, 1e-6), (2, 1e-7, 1e-6)])
def test_large_workload_like_solve_matches_golden(prec, conv, tol):
    """A scaled-down instance of the large mixed-precision workload: o=16, v=160, X=480, seed 2, B x 0.05,
    5 canonical roots, the ladder assembled from the factor in every application (that workload's form),
    FP64 and FP32 / BF16 sigma with the FP64 restart, against the oracle's golden (conv 1e-9)."""
    g = _golden("large-like-o16v160x480_s0.05")
    eo, ev, B = synth.make_instance(g["nocc"], g["nvir"], g["naux"], g["seed"], scale=g["scale"])
    print("large-like solve precision %d" % prec, flush=True)
    o = adc.adc3_default_opts()
    o.ladder, o.precision = 2, prec
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 5, 0.0, 0.0, conv, opts=o)
    assert st == adc.ADC3_OK
    err = np.abs(roots - np.array(g["roots"]))
    print("root errors vs the oracle", err)
    assert err.max() < tol
    assert all(abs(r["omega"] - w) <= r["err_bound"] + 1e-12 for r, w in zip(reps, g["roots"]))


def test_batched_workload_instances_match_goldens():
    """Instances of the ragged batched workload (literal scale, 8 roots, conv 1e-6) with stored oracle roots:
    the lockstep batch in the workload's configuration (FP32 ladder, sigma graphs, two slots)."""
    import glob
    import os
    files = sorted(glob.glob(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch-seed*.json")))
    assert len(files) >= 3
    gold = [_golden(os.path.basename(f)[:-5]) for f in files]
    inst = []
    for gd in gold:
        eo, ev, B = synth.batch_instance(gd["seed"])
        inst.append(dict(eps_occ=dev(eo), eps_vir=dev(ev), B=dev(B), nroots=8, conv=1e-6))
    print("batched goldens: %d instances" % len(inst), flush=True)
    o = _opts(precision=1, sigma_graphs=1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        roots, reps, sts, st = adc.adc3_ea_solve_batched(inst, opts=o, nstreams=2)
    torch.cuda.synchronize()
    assert st == 0 and all(s == 0 for s in sts)
    for gd, r in zip(gold, roots):
        ref = np.array(gd["roots"])
        assert np.all(np.abs(r - ref) <= 1e-6 + 1e-12 * np.abs(ref)), (gd["seed"], np.abs(r - ref).max())
