"""Write FP64 oracle references for the seven-cell workload (4096 instances:
hexagonal layout with 500 m inter-site distance, per instance M in
{16,32,64,128}, N in {1,2,4}, d = min(N,2), 2..12 users per cell, path loss
128.1 + 37.6 log10(d_km) dB with 8 dB shadowing, noise -174 dBm/Hz over
10 MHz, 46 dBm per BS).

Calls only the CPU oracle, on a fixed sample of the batch (every 8th
instance: 512 of 4096):
  * WMMSE (Algorithm 2, reference mode: stop at relative WSR change <= 1e-6 or
    after 500 iterations) on all 512 sampled instances, the 99 % target of
    the instances/s count;
  * A-MMMSE (Algorithm 3, T = 100, eps1 = 0.1, T_c = 3, default step rule) on
    the first 16 sampled instances of each tile-shape class of the GPU
    kernel (the widest per-cell precoder block n = max_c U_c d: n <= 16,
    16 < n <= 32, n > 32): final WSR (bits), stage-switch iteration and the
    WSR trace, against which the float solve of the whole batch is scored.

    python tests/golden/make_hexcell_reference.py [--workers 8] [--part wmmse|ammmse|all]
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

OUT = os.path.join(HERE, "oracle_ref_hexcell7_b4096.json")
STRIDE = 8
PER_CLASS = 16


def shape_class(inst):
    n = max(int(u) * int(inst["d"]) for u in inst["cell_users"])
    return 0 if n <= 16 else (1 if n <= 32 else 2)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--part", default="all", choices=["all", "wmmse", "ammmse"])
    a = ap.parse_args()
    b = synth.hexcell_batch(4096)
    index = list(range(0, b.batch, STRIDE))
    insts = [b.instance(i) for i in index]
    out = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            out = json.load(f)
    out.update(workload=b.name, seeds="synth.hexcell_batch(4096)",
               sample=f"every {STRIDE}th instance", index=index)
    if a.part in ("all", "ammmse"):
        t0 = time.time()
        pick, count = [], [0, 0, 0]
        for k, inst in enumerate(insts):
            c = shape_class(inst)
            if count[c] < PER_CLASS:
                pick.append(k)
                count[c] += 1
        am = O.solve_batch([insts[k] for k in pick], "ammmse", workers=a.workers, iters=100)
        out["ammmse"] = dict(
            algorithm="A-MMMSE (Algorithm 3), FP64, T=100, eps1=0.1, T_c=3, default step rule",
            index=[index[k] for k in pick], shape_class=[shape_class(insts[k]) for k in pick],
            wsr=[float(r["wsr"]) for r in am], switch_iter=[int(r["switch_iter"]) for r in am],
            trace=[[float(x) for x in r["trace"]] for r in am], seconds=time.time() - t0)
        print("ammmse", f"{time.time() - t0:.0f}s", flush=True)
    if a.part in ("all", "wmmse"):
        t0 = time.time()
        wm = O.solve_batch(insts, "wmmse", workers=a.workers, max_iters=500, eps=1e-6,
                           mode="reference")
        out["wmmse"] = dict(algorithm="WMMSE (Algorithm 2), FP64 reference mode",
                            stop="relative WSR change <= 1e-6 or 500 iterations",
                            wsr=[float(r["wsr"]) for r in wm],
                            iters=[int(r["iters"]) for r in wm], seconds=time.time() - t0)
        print("wmmse", f"{time.time() - t0:.0f}s", flush=True)
    out["workers"] = a.workers
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(OUT)


if __name__ == "__main__":
    main()
