"""Mixed precision (bfloat16 channel products with float accumulation, float
refinement pass) against the FP64 oracle.

Workload: the M=256 Rayleigh batch (64 users, N=d=2, P=20 dB, sigma2=1,
alpha ~ U[0.5, 1.5]); the oracle's A-MMMSE WSR after T=100 iterations for the
first 16 instances is stored in tests/golden (written by
tests/golden/make_large_reference.py, which calls only the oracle).

Bars (relative WSR error against the FP64 oracle, per instance):
  * bfloat16 products throughout (no refinement): <= 1e-2, both for the WSR
    the solver reports and for the oracle's WSR of the returned precoder;
  * with the float refinement pass (last 10 of 100 iterations): <= 1e-4;
    the reported WSR is then the float evaluation of the returned precoder
    (checked against the oracle's evaluation to 1e-6).
"""
import json
import os

import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth
import oracle as O

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "oracle_ref_rayleigh_m256u64n2d2_b512.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def large16():
    with open(GOLD) as f:
        ref = json.load(f)["ammmse"]
    b = synth.rayleigh_large(512).subset(np.arange(len(ref["index"])))
    return b, np.array(ref["wsr"]), np.array(ref["switch_iter"])


def oracle_wsr_of(batch, V):
    """FP64 oracle WSR (bits) of the returned precoders, per instance."""
    out = []
    for i in range(batch.batch):
        inst = batch.instance(i)
        prob = O.from_instance(inst)
        off = int(batch.v_off[i])
        blocks = []
        for c in range(inst["C"]):
            n = inst["M"] * inst["cell_users"][c] * inst["d"]
            blocks.append(V[off: off + n].reshape(inst["M"], -1))
            off += n
        out.append(O.wsr_bits(prob, O.split_v(prob, blocks)))
    return np.array(out)


def _solve(b, refine):
    opts = ammse.Options(precision=ammse.PREC_BF16, max_iters=100, refine_iters=refine)
    return ammse.solve(b, opts)


def test_bf16_before_refinement(large16):
    b, ref, sw = large16
    res = _solve(b, 0)
    assert (res.status == 0).all()
    np.testing.assert_array_equal(res.switch_iter, sw)
    rep = np.abs(res.wsr - ref) / ref
    true = np.abs(oracle_wsr_of(b, res.V) - ref) / ref
    say(f"bf16, no refinement: reported err max {rep.max():.2e}, true err max {true.max():.2e}")
    assert rep.max() <= 1e-2 and true.max() <= 1e-2


def test_bf16_after_refinement(large16):
    b, ref, sw = large16
    res = _solve(b, 10)
    assert (res.status == 0).all()
    np.testing.assert_array_equal(res.switch_iter, sw)
    tw = oracle_wsr_of(b, res.V)
    rep = np.abs(res.wsr - ref) / ref
    true = np.abs(tw - ref) / ref
    say(f"bf16 + 10 float iterations: reported err max {rep.max():.2e}, true err max "
        f"{true.max():.2e}, evaluation err {np.abs(res.wsr - tw).max() / tw.min():.2e}")
    assert np.abs(res.wsr - tw).max() <= 1e-6 * tw.min()
    assert rep.max() <= 1e-4 and true.max() <= 1e-4


def test_fp32_general_on_large(large16):
    b, ref, sw = large16
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP32, max_iters=100))
    err = np.abs(res.wsr - ref) / ref
    say(f"fp32: err max {err.max():.2e}")
    assert (res.status == 0).all() and err.max() <= 1e-4


def test_bf16_all_refined_equals_fp32():
    """refine_iters >= max_iters: no bfloat16 product is taken, so the run is
    the float general-kernel run bit for bit."""
    b = synth.rayleigh_large(8, seed=24999)
    a = ammse.solve(b, ammse.Options(precision=ammse.PREC_BF16, max_iters=30, refine_iters=30),
                    want_trace=True)
    f = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP32, max_iters=30,
                                     path=ammse.PATH_GENERAL), want_trace=True)
    np.testing.assert_array_equal(a.trace, f.trace)
    np.testing.assert_array_equal(a.V, f.V)


def test_bf16_ragged_multicell():
    """Uneven multi-cell instances (7-cell layout), 60 iterations, last 10 in
    float: no failure flag; the reported WSR is the float evaluation of the
    returned precoder (checked against the oracle's evaluation); every BS
    meets its budget; the whole WSR trace (same stage switch as the FP64
    oracle) within 5e-2 of the oracle's.  This layout's path-loss spread
    makes its trajectories amplify the ~4e-3 rounding of bfloat16 products
    more than the Rayleigh workloads do: measured gaps 2.3e-3 to 2.2e-2, so the
    1e-2 bar of the M=256 workload is not met on every instance here and the
    bar of this test is 5e-2."""
    b = synth.hexcell_batch(8, seed=23999)
    T = 60
    refs = []
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        refs.append(O.ammmse(prob, O.split_v(prob, inst["V0"]), T))
    fs = np.array([r["switch_iter"] if r["switch_iter"] >= 1 else T + 1 for r in refs], np.int32)
    mixed = ammse.solve(b, ammse.Options(precision=ammse.PREC_BF16, max_iters=T, refine_iters=10),
                        want_trace=True, force_switch=fs)
    assert (mixed.status == 0).all()
    tw = oracle_wsr_of(b, mixed.V)
    ev = np.abs(mixed.wsr - tw) / tw
    say(f"hexcell bf16: evaluation err max {ev.max():.2e}")
    assert ev.max() <= 1e-5
    for i in range(b.batch):
        inst = b.instance(i)
        off = int(b.v_off[i])
        for c in range(inst["C"]):
            n = inst["M"] * inst["cell_users"][c] * inst["d"]
            p_c = float(np.sum(np.abs(mixed.V[off: off + n]) ** 2))
            assert p_c <= b.P[b.bs_off[i] + c] * (1 + 1e-5), (i, c)
            off += n
        gap = np.abs(mixed.trace[i] - refs[i]["trace"]) / refs[i]["trace"]
        say(f"instance {i}: max rel gap to the oracle {gap.max():.2e} (final {gap[-1]:.2e})")
        assert gap.max() <= 5e-2, i
