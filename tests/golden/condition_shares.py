"""Write condition_shares.json: the share of pixels the oracle's conditioning
classifier excludes, per benchmark workload (whole frames), under two
settings of its jittered re-traces:

  survey   relative jitter 2^-23 (one FP32 ulp), 4 re-traces, spread 1e-5;
  current  relative jitter 2^-21 (four ulps), 8 re-traces, spread 2.5e-5,
           the setting the GPU parity tests use (oracle.JITTER, COND_RUNS,
           COND_SPREAD).

Also the share of ID-grazing pixels (primary decision margin below 1e-6).
Calls only the oracle and the seeded scene generator.  Run from the
repository root:  python tests/golden/condition_shares.py
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import scenegen  # noqa: E402

SETTINGS = {"survey": dict(jitter=2.0 ** -23, runs=4, spread=1e-5),
            "current": dict(jitter=oracle.JITTER, runs=oracle.COND_RUNS,
                            spread=oracle.COND_SPREAD)}


def main():
    oracle.build()
    out = {"settings": {}}
    bases = {}
    for name, st in SETTINGS.items():
        res = {}
        for i in (0, 1, 2, 4):
            wl = scenegen.make_workload(i)
            if i not in bases:
                bases[i] = oracle.render(wl.scene, wl.camera, wl.W, wl.H, wl.depth)
            base = bases[i]
            t0 = time.time()
            ok = oracle.condition(wl.scene, wl.camera, wl.W, wl.H, wl.depth, base=base, **st)
            res[wl.name] = {"pixels": int(ok.size),
                            "ill_conditioned": float((~ok).mean()),
                            "grazing": float((base.margin < oracle.GRAZING).mean())}
            print(name, wl.name, res[wl.name], "%.1f s" % (time.time() - t0), flush=True)
        out["settings"][name] = dict(st, workloads=res)
    with open(os.path.join(HERE, "condition_shares.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
