"""The ladder term assembled from the DF factor in every application (adc3_opts.ladder = 2,
adc3_ladder_apply) against the FP64 oracle: the ladder alone (every row at small sizes, with one
and with several auxiliary chunks; sampled rows at the o=40, v=600, X=150 shape of the large
workload after NAF), sigma and roots of contexts and solves that use it, and the coupling build cut
into chunks of the first virtual index.

Tolerances: FP64 as elsewhere (relative 1e-12 of the largest element for the ladder alone, 1e-11 for
sigma, 1e-8 Eh for roots).  FP32 operands (inputs and the intermediate rounded to 24 bits, FP32
accumulation over K = X v terms): 2e-5 of the largest element.  BF16 operands (8 bits): 3e-2.
Mixed-precision roots: 1e-6 Eh after the FP64 restart.
"""
import numpy as np
import pytest

import synth
from oracle import ssfno
from oracle.adc_cs import Problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2511_05897_amd as adc  # noqa: E402

LP_TOL = {0: 1e-12, 1: 2e-5, 2: 3e-2}


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# (v, X, rows, seed): ragged shapes (scalar loads), vector-friendly ones, a row count past one tile
LADDER_SMALL = [(7, 5, 3, 1), (9, 13, 17, 2), (16, 24, 20, 3), (40, 60, 37, 4), (24, 9, 130, 5)]


@pytest.mark.parametrize("case", LADDER_SMALL, ids=lambda c: "v%dx%dm%d" % c[:3])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_ladder_apply_small(case, prec):
    v, X, M, seed = case
    eo, ev, B = synth.make_instance(2, v, X, seed, scale=0.5)
    P = Problem(eo, ev, B)
    Z = np.random.default_rng(seed).standard_normal((M, v, v))
    ref = P.vvvv_apply(Z)
    Bd, Zd = dev(P.Bvv), dev(Z)
    eb = 8 if prec == 0 else 4 if prec == 1 else 2
    one = adc.adc3_ladder_workspace_bytes(v, X, M, prec) + 512
    for nbytes in (one, one + 2 * M * v * v * eb, one + X * M * v * v * eb):  # 1, 3 and all X per chunk
        out = host(adc.adc3_ladder_apply(Bd, Zd, precision=prec, workspace_bytes=nbytes))
        assert relerr(out, ref) < LP_TOL[prec], (nbytes, relerr(out, ref))


def test_ladder_apply_rejects_bad_arguments():
    eo, ev, B = synth.make_instance(2, 8, 6, 1)
    P = Problem(eo, ev, B)
    Bd, Zd = dev(P.Bvv), dev(np.ones((3, 8, 8)))
    with pytest.raises(adc.ADCError) as e:
        adc.adc3_ladder_apply(Bd, Zd, workspace_bytes=adc.adc3_ladder_workspace_bytes(8, 6, 3, 0) - 8)
    assert e.value.status == adc.ADC3_ENOMEM
    with pytest.raises(adc.ADCError) as e:
        adc.adc3_ladder_apply(Bd, Zd, precision=3)
    assert e.value.status == adc.ADC3_EINVAL


@pytest.fixture(scope="module")
def large_shape():
    """v=600, X=150 (the large workload's NAF-kept size), 200 rows (5 vectors x 40 occupied); the
    oracle's ladder of rows 0, 77 and 199."""
    v, X, M = 600, 150, 200
    eo, ev, B = synth.make_instance(1, v, X, 2)
    P = Problem(eo, ev, B)
    del B
    Z = np.random.default_rng(9).standard_normal((M, v, v))
    rows = (0, 77, 199)
    return P.Bvv, Z, rows, [P.vvvv_apply(Z[m:m + 1])[0] for m in rows]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_ladder_apply_large_workload_shape_sampled_rows(large_shape, prec):
    """8 GB of intermediate (13 auxiliary chunks)."""
    Bvv, Z, rows, refs = large_shape
    M, v, X = Z.shape[0], Z.shape[1], Bvv.shape[0]
    out = adc.adc3_ladder_apply(dev(Bvv), dev(Z), precision=prec,
                                workspace_bytes=adc.adc3_ladder_workspace_bytes(v, X, M, prec) + (8 << 30))
    for m, ref in zip(rows, refs):
        got = host(out[m])
        assert relerr(got, ref) < LP_TOL[prec], (m, relerr(got, ref))
    del out
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def full_large_shape():
    """The large workload itself: o=40, v=600, X=1800, seed 2 (its virtual block Bvv, 5.2 GB), 200 rows
    (5 vectors x 40 occupied).  The oracle samples rows a of chosen vectors m: 9 x 600 elements."""
    eo, ev, B = synth.make_instance(40, 600, 1800, 2)
    Bvv = np.ascontiguousarray(B[:, 40:, 40:])
    del B
    Z = np.random.default_rng(13).standard_normal((200, 600, 600))
    from oracle.adc_cs import ladder_rows
    ms, aa = (0, 117, 199), (0, 311, 599)
    refs = {m: ladder_rows(Bvv, Z[m], aa) for m in ms}
    return Bvv, Z, ms, aa, refs


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_ladder_apply_full_large_workload_sampled(full_large_shape, prec):
    """sum_Q B^Q Z B^Q at v=600, X=1800, 200 rows (the assembled ladder of the large workload's canonical
    basis), 8 GB of intermediate per chunk; sampled elements against the oracle in all three precisions."""
    Bvv, Z, ms, aa, refs = full_large_shape
    M, v, X = Z.shape[0], Z.shape[1], Bvv.shape[0]
    print("assembled ladder v=%d X=%d rows=%d precision %d" % (v, X, M, prec), flush=True)
    Bd = dev(Bvv)
    out = adc.adc3_ladder_apply(Bd, dev(Z), precision=prec,
                                workspace_bytes=adc.adc3_ladder_workspace_bytes(v, X, M, prec) + (8 << 30))
    scale = max(np.abs(r).max() for r in refs.values())
    for m in ms:
        got = host(out[m])[list(aa)]
        err = np.abs(got - refs[m]).max() / scale
        assert err < LP_TOL[prec], (m, err)
    del out, Bd
    torch.cuda.empty_cache()


SMALL = [(3, 7, 15, 3, 0.5), (2, 9, 20, 4, 1.0), (5, 17, 40, 5, 0.3)]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "o%dv%dx%d" % c[:3])
def test_sigma_assembled_ladder_matches_oracle(case):
    o, v, X, seed, sc = case
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=sc)
    P = Problem(eo, ev, B)
    r = np.random.default_rng(11).standard_normal((19, P.dim()))  # a full pass of 16 and a ragged one
    ref = P.sigma(r, 3)
    ctx = adc.Context(dev(eo), dev(ev), dev(B), 3, ladder=2)
    assert relerr(host(ctx.sigma(dev(r))), ref) < 1e-11
    assert relerr(host(ctx.diagonal()), P.diagonal(3)) < 1e-11
    ctx.close()
    for prec in (1, 2):
        ctx = adc.Context(dev(eo), dev(ev), dev(B), 3, precision=prec, ladder=2)
        e = relerr(host(ctx.sigma(dev(r[:5]), precision=prec)), ref[:5])
        assert e < (1e-5 if prec == 1 else 2e-2), (prec, e)
        ctx.close()


def test_coupling_build_in_chunks_matches_oracle():
    """A chunk budget of 3 o v^2 elements cuts the coupling build into chunks of 3 virtuals (and the
    assembled ladder into one auxiliary function per chunk): intermediates and sigma unchanged."""
    o, v, X, seed = 3, 10, 24, 8
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=0.5)
    P = Problem(eo, ev, B)
    prev = adc.adc3_set_chunk_elems(3 * o * v * v)
    try:
        for level, ladder in ((2, 0), (3, 1), (3, 2)):
            ctx = adc.Context(dev(eo), dev(ev), dev(B), level, ladder=ladder)
            Uz = host(ctx.intermediate(1)).reshape(v, o, v, v)
            assert relerr(Uz, P.coupling_z(level)) < 1e-11
            assert relerr(host(ctx.intermediate(0)).reshape(v, v), P.m11(level)) < 1e-11
            r = np.random.default_rng(2).standard_normal((4, P.dim()))
            assert relerr(host(ctx.sigma(dev(r))), P.sigma(r, level)) < 1e-11
            ctx.close()
    finally:
        adc.adc3_set_chunk_elems(prev)
    assert adc.adc3_set_chunk_elems(0) == prev


def test_solve_assembled_ladder_matches_oracle():
    # canonical ADC(3), tiny dense instance: full diagonalisation of the oracle's matrix
    p, eo, ev, B = synth.preset("tiny-dense")
    ref = np.linalg.eigvalsh(Problem(eo, ev, B).dense(3))[:3]
    o = adc.adc3_default_opts()
    o.ladder = 2
    roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 0.0, 0.0, 1e-8, opts=o)
    assert st == adc.ADC3_OK and np.abs(roots - ref).max() < 1e-8
    # SS-FNO + NAF pipeline (truncation active) against the oracle pipeline, FP64 and mixed precision
    eo, ev, B = synth.make_instance(3, 10, 24, 8, scale=0.3)
    refp = ssfno.run(eo, ev, B, 3, 1e-4, 1e-2, 1e-9)
    for prec, tol in ((0, 1e-8), (1, 1e-6), (2, 1e-6)):
        o.precision = prec
        roots, reps, st = adc.adc3_ea_solve(dev(eo), dev(ev), dev(B), 3, 1e-4, 1e-2, 1e-8, opts=o)
        assert st == adc.ADC3_OK
        assert [r["nvir_kept"] for r in reps] == list(refp["nvir_kept"])
        assert [r["naux_kept"] for r in reps] == list(refp["naux_kept"])
        assert np.abs(roots - refp["roots"]).max() < tol, prec


def test_sigma_graph_replays_with_assembled_ladder():
    """Sigma passes with the assembled ladder captured into HIP graphs and replayed (FP64 and BF16 contexts),
    against eager passes, with the program's own eager work between replays."""
    o, v, X, seed = 3, 16, 24, 6
    eo, ev, B = synth.make_instance(o, v, X, seed, scale=0.5)
    P = Problem(eo, ev, B)
    rng = np.random.default_rng(4)
    rs = [rng.standard_normal((nv, P.dim())) for nv in (3, 17)]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for prec in (0, 2):
            ctx = adc.Context(dev(eo), dev(ev), dev(B), 3, precision=prec, ladder=2)
            eager = [host(ctx.sigma(dev(r), precision=prec)) for r in rs]
            for r, e in zip(rs, eager):
                assert relerr(e, P.sigma(r, 3)) < (1e-11 if prec == 0 else 2e-2)
            ctx.set_sigma_graphs(True)
            for rep in range(3):
                for r, e in zip(rs, eager):
                    out = host(ctx.sigma(dev(r), precision=prec))
                    assert np.abs(out - e).max() <= 1e-14 * np.abs(e).max(), (prec, rep)
                    x = torch.randn(1000, device="cuda", dtype=torch.float64)
                    (x * 2.0).sum().item()
            ctx.close()
    torch.cuda.synchronize()
