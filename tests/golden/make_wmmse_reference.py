"""Write FP64 oracle references of the Rayleigh sweep workload (M=64, 16
users, N=d=4, P in {0,10,20,30} dB, 256 instances per SNR).

Calls only the CPU oracle:
  * WMMSE (Algorithm 2, reference mode: dual bisection to relative width
    1e-12, stop at relative WSR change <= 1e-6 or after 500 iterations) on
    every instance: final WSR (bits) and iteration counts.  The benchmark
    counts a GPU solve as successful when its WSR reaches 99 % of this value.
  * A-MMMSE (Algorithm 3, T = 100, eps1 = 0.1, T_c = 3, default step rule) on
    8 instances per SNR spread over the batch: final WSR, stage-switch
    iteration and WSR trace, against which sampled instances of the float
    solve of the whole batch are scored.

    python tests/golden/make_wmmse_reference.py [--workers 8] [--part wmmse|ammmse|all]
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


AMMMSE_INDEX = [k * 256 + j for k in range(4) for j in (3, 37, 70, 101, 140, 177, 211, 250)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--part", default="all", choices=["all", "wmmse", "ammmse"])
    a = ap.parse_args()
    b = synth.rayleigh_sweep(B_per_p=256)
    insts = [b.instance(i) for i in range(b.batch)]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    if a.part in ("all", "wmmse"):
        t0 = time.time()
        res = O.solve_batch(insts, "wmmse", workers=a.workers, max_iters=500, eps=1e-6,
                            mode="reference")
        out.update(workload=b.name, algorithm="WMMSE (Algorithm 2), FP64 reference mode",
                   stop="relative WSR change <= 1e-6 or 500 iterations; bisection rel. width 1e-12",
                   seeds="synth.rayleigh_sweep(B_per_p=256)",
                   wsr=[float(r["wsr"]) for r in res], iters=[int(r["iters"]) for r in res],
                   P=[float(x) for x in b.P], seconds=time.time() - t0, workers=a.workers)
    if a.part in ("all", "ammmse"):
        t0 = time.time()
        am = O.solve_batch([insts[i] for i in AMMMSE_INDEX], "ammmse", workers=a.workers,
                           iters=100)
        out["ammmse"] = dict(
            algorithm="A-MMMSE (Algorithm 3), FP64, T=100, eps1=0.1, T_c=3, default step rule",
            index=AMMMSE_INDEX, wsr=[float(r["wsr"]) for r in am],
            switch_iter=[int(r["switch_iter"]) for r in am],
            trace=[[float(x) for x in r["trace"]] for r in am], seconds=time.time() - t0)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT)


if __name__ == "__main__":
    main()
