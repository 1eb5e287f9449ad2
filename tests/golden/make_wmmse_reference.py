"""Write the FP64 WMMSE reference WSR of the Rayleigh sweep workload.

Calls only the CPU oracle (WMMSE, Algorithm 2, reference mode: dual bisection
to relative width 1e-12, stop at relative WSR change <= 1e-6 or after 500
iterations) on every instance of the seeded workload (M=64, 16 users, N=d=4,
P in {0,10,20,30} dB, 256 instances per SNR) and stores the final WSR (bits)
and iteration counts as JSON.  The benchmark counts a GPU solve as
successful when its WSR reaches 99 % of this value.

    python tests/golden/make_wmmse_reference.py [--workers 8]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2510_20507_amd import synth  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "wmmse_ref_rayleigh_sweep4x256.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    b = synth.rayleigh_sweep(B_per_p=256)
    insts = [b.instance(i) for i in range(b.batch)]
    t0 = time.time()
    res = O.solve_batch(insts, "wmmse", workers=a.workers, max_iters=500, eps=1e-6,
                        mode="reference")
    out = dict(workload=b.name, algorithm="WMMSE (Algorithm 2), FP64 reference mode",
               stop="relative WSR change <= 1e-6 or 500 iterations; bisection rel. width 1e-12",
               seeds="synth.rayleigh_sweep(B_per_p=256)",
               wsr=[float(r["wsr"]) for r in res], iters=[int(r["iters"]) for r in res],
               P=[float(x) for x in b.P], seconds=time.time() - t0, workers=a.workers)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT, f"{out['seconds']:.0f}s")


if __name__ == "__main__":
    main()
