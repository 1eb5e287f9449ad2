"""Write FP64 oracle references for the M=256 Rayleigh workload (512
instances: M=256, 64 users, N=d=2, P=20 dB, sigma2=1, alpha ~ U[0.5, 1.5]).

Calls only the CPU oracle:
  * A-MMMSE (Algorithm 3, T=100, eps1=0.1, T_c=3, default step rule) on the
    first 16 instances:
    final WSR (bits) and stage-switch iteration, against which the mixed
    bfloat16 / float solves are scored;
  * WMMSE (Algorithm 2, reference mode: stop at relative WSR change <= 1e-6
    or 500 iterations) on all 512 instances, the 99 % target of the
    instances/s count.

    python tests/golden/make_large_reference.py [--workers 8] [--part wmmse|ammmse|all]
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

OUT = os.path.join(HERE, "oracle_ref_rayleigh_m256u64n2d2_b512.json")
N_AMMMSE = 16


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--part", default="all", choices=["all", "wmmse", "ammmse"])
    a = ap.parse_args()
    b = synth.rayleigh_large(512)
    insts = [b.instance(i) for i in range(b.batch)]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    out.update(workload=b.name, seeds="synth.rayleigh_large(512)")
    t0 = time.time()
    if a.part in ("all", "ammmse"):
        am = O.solve_batch(insts[:N_AMMMSE], "ammmse", workers=a.workers, iters=100)
        out["ammmse"] = dict(
            algorithm="A-MMMSE (Algorithm 3), FP64, T=100, eps1=0.1, T_c=3, default step rule",
            index=list(range(N_AMMMSE)), wsr=[float(r["wsr"]) for r in am],
            switch_iter=[int(r["switch_iter"]) for r in am],
            trace=[[float(x) for x in r["trace"]] for r in am], seconds=time.time() - t0)
    t1 = time.time()
    if a.part in ("all", "wmmse"):
        wm = O.solve_batch(insts, "wmmse", workers=a.workers, max_iters=500, eps=1e-6,
                           mode="reference")
        out["wmmse"] = dict(algorithm="WMMSE (Algorithm 2), FP64 reference mode",
                            stop="relative WSR change <= 1e-6 or 500 iterations",
                            wsr=[float(r["wsr"]) for r in wm],
                            iters=[int(r["iters"]) for r in wm], seconds=time.time() - t1)
    out["workers"] = a.workers
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
