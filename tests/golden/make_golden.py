"""Write the stored expected values of the full-size workloads.  Calls only oracle/ and synth.

    python tests/golden/make_golden.py ssfno-o20v200x600 [scale] [conv]
    python tests/golden/make_golden.py instance NAME NOCC NVIR NAUX SEED SCALE NROOTS CONV
    python tests/golden/make_golden.py batch SEED [NROOTS] [CONV]

Writes tests/golden/<workload>[_s<scale>].json with the corrected roots, the
uncorrected ADC(3) roots, the canonical and truncated ADC(2) roots and the kept
virtual/auxiliary counts of the SS-FNO/NAF pipeline (Sec. "Computational
Details", steps 2-4f), computed by the FP64 oracle with Davidson conv 1e-8 (default) or
the given conv (the literal scale, |omega| ~ 1e6 Eh, cannot reach 1e-8 in FP64).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import ssfno  # noqa: E402


def canonical(name, eo, ev, B, nroots, conv, meta):
    """Canonical EA-ADC(3) roots (no truncation) of one instance, FP64 oracle Davidson."""
    t0 = time.time()
    r = ssfno.run(eo, ev, B, nroots, 0.0, 0.0, conv, dense_limit=0)
    out = dict(meta, name=name, oracle_conv=conv, seconds=time.time() - t0, nroots=nroots,
               roots=[float(x) for x in r["roots"]], converged=bool(r["converged"]))
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    if sys.argv[1] == "instance":
        name = sys.argv[2]
        o, v, X, seed = (int(x) for x in sys.argv[3:7])
        scale, nroots, conv = float(sys.argv[7]), int(sys.argv[8]), float(sys.argv[9])
        eo, ev, B = synth.make_instance(o, v, X, seed, scale=scale)
        canonical(name, eo, ev, B, nroots, conv, dict(nocc=o, nvir=v, naux=X, seed=seed, scale=scale))
        return
    if sys.argv[1] == "batch":
        seed = int(sys.argv[2])
        nroots = int(sys.argv[3]) if len(sys.argv) > 3 else 8
        conv = float(sys.argv[4]) if len(sys.argv) > 4 else 1e-6
        rng, o, v, X = synth.batch_shapes(seed)
        eo, ev, B = synth.batch_instance(seed)
        canonical("batch-seed%d" % seed, eo, ev, B, nroots, conv, dict(nocc=o, nvir=v, naux=X, seed=seed, scale=1.0))
        return
    name = sys.argv[1]
    scale = float(sys.argv[2]) if len(sys.argv) > 2 else 1.0
    conv = float(sys.argv[3]) if len(sys.argv) > 3 else 1e-8
    p, eo, ev, B = synth.preset(name, scale=scale)
    t0 = time.time()
    r = ssfno.run(eo, ev, B, p["nroots"], p["fno_thresh"], p["naf_thresh"], conv)
    out = {"workload": name, "scale": scale, "oracle_conv": conv, "seconds": time.time() - t0,
           "roots": [float(x) for x in r["roots"]],
           "omega_uncorr": [float(x) for x in r["omega_uncorr"]],
           "omega_adc2_can": [float(x) for x in r.get("omega_adc2_can", [])],
           "omega_adc2_fno": [float(x) for x in r.get("omega_adc2_fno", [])],
           "nvir_kept": [int(x) for x in r["nvir_kept"]], "naux_kept": [int(x) for x in r["naux_kept"]]}
    tag = name if scale == 1.0 else "%s_s%g" % (name, scale)
    with open(os.path.join(HERE, tag + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
