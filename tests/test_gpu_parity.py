"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances:
  * FP64 path: WSR trajectories agree to 1e-9 relative per iteration and the
    precoders to 1e-7 of their norm (only rounding order differs).
  * FP32 path: WSR trajectory, final WSR included, within 1e-4 relative of the
    FP64 oracle at every iteration.
The stage switch is an integer decided by comparing a floating-point change
with eps1; where the two sides decide differently on a borderline case the
GPU run is repeated with the oracle's switch iteration forced, so that both
follow the same branch of Algorithm 3.
"""
import math

import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth
import oracle as O
from instances import instance, random_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def say(*a):
    print(*a, flush=True)


def oracle_runs(batch, idx, **kw):
    out = []
    for i in idx:
        inst = batch.instance(int(i))
        prob = O.from_instance(inst)
        out.append(O.ammmse(prob, O.split_v(prob, inst["V0"]), **kw))
    return out


def v_blocks(batch, V, i):
    """Per-BS blocks of instance i from a flat complex vector."""
    inst = batch.instance(i)
    off = int(batch.v_off[i])
    out = []
    for c in range(inst["C"]):
        n = inst["M"] * inst["cell_users"][c] * inst["d"]
        out.append(V[off: off + n].reshape(inst["M"], -1))
        off += n
    return out


def compare_wsr(batch, res, refs, idx, opts, tol, force_retry=True):
    """Compare final WSR; re-run borderline stage switches with the oracle's value."""
    bad = []
    for k, i in enumerate(idx):
        ref = refs[k]
        if res.switch_iter[i] != ref["switch_iter"]:
            bad.append(k)
            continue
        err = abs(res.wsr[i] - ref["wsr"]) / abs(ref["wsr"])
        assert err <= tol, (i, res.wsr[i], ref["wsr"], err)
    if bad and force_retry:
        sub = batch.subset([idx[k] for k in bad])
        fs = np.array([refs[k]["switch_iter"] for k in bad], np.int32)
        r2 = ammse.solve(sub, opts, force_switch=fs)
        for j, k in enumerate(bad):
            err = abs(r2.wsr[j] - refs[k]["wsr"]) / abs(refs[k]["wsr"])
            assert err <= tol, (idx[k], r2.wsr[j], refs[k]["wsr"], err)
    return len(bad)


def compare_traces(batch, res, refs, idx, opts, tol):
    """Whole WSR trajectories (WSR(V^0) .. WSR(V^T), the final WSR included)
    against the oracle at every iteration; borderline stage switches are re-run
    with the oracle's switch."""
    for k, i in enumerate(idx):
        ref = refs[k]
        tr = res.trace[i]
        if res.switch_iter[i] != ref["switch_iter"]:
            r2 = ammse.solve(batch.subset([i]), opts, want_trace=True,
                             force_switch=np.array([ref["switch_iter"]], np.int32))
            tr = r2.trace[0]
        rt = np.asarray(ref["trace"])
        err = np.abs(tr - rt) / np.abs(rt)
        assert err.max() <= tol, (i, int(err.argmax()), float(err.max()))


def golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# FP64: iterate-level parity
# ---------------------------------------------------------------------------

def test_fp64_single_small_200_iterations():
    b = synth.single_small()
    say("case: single_small fp64 T=200")
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=200), want_trace=True)
    ref = oracle_runs(b, [0], iters=200)[0]
    assert res.status[0] == 0
    assert res.switch_iter[0] == ref["switch_iter"]
    np.testing.assert_allclose(res.trace[0], ref["trace"], rtol=1e-9)
    Vg = v_blocks(b, res.V, 0)[0]
    Vr = np.concatenate(ref["V_blocks"] if "V_blocks" in ref else
                        O.join_v(O.from_instance(b.instance(0)), ref["V"]), axis=1)
    assert np.linalg.norm(Vg - Vr) <= 1e-7 * np.linalg.norm(Vr)
    assert res.iters[0] == 200


def _ragged_batch():
    insts = [
        random_instance(101, M=5, cell_users=[2, 1], N=2, d=1, P=[2.0, 3.0], sigma2=0.5,
                        alpha_range=(0.5, 1.5)),
        random_instance(102, M=7, cell_users=[1, 0, 2], N=3, d=2, P=[1.0, 4.0, 2.0]),
        random_instance(103, M=70, cell_users=[5], N=1, d=1, P=10.0, alpha_range=(0.5, 1.5)),
        random_instance(104, M=16, cell_users=[3, 3], N=4, d=4, P=[5.0, 5.0], sigma2=0.2),
        random_instance(105, M=66, cell_users=[20], N=4, d=3, P=30.0, alpha_range=(0.5, 1.5)),
        random_instance(106, M=3, cell_users=[2], N=2, d=2, P=1.0),
    ]
    return synth.pack(insts, name="ragged")


def test_fp64_ragged_shapes_iterates():
    """Uneven shapes spanning several 64-wide tiles with ragged tails, empty
    cells, N = 1..4, d < N, M < N*U, in one launch."""
    b = _ragged_batch()
    T = 60
    refs = oracle_runs(b, range(b.batch), iters=T)
    fs = np.array([r["switch_iter"] for r in refs], np.int32)
    say("case: ragged fp64 T=60", b.batch)
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=T), want_trace=True,
                      force_switch=fs)
    for i, ref in enumerate(refs):
        assert res.status[i] == 0, i
        np.testing.assert_allclose(res.trace[i], ref["trace"], rtol=1e-9, err_msg=str(i))
        Vg = np.concatenate(v_blocks(b, res.V, i), axis=1)
        Vr = np.concatenate(ref["V_blocks"] if "V_blocks" in ref else
                            O.join_v(O.from_instance(b.instance(i)), ref["V"]), axis=1)
        assert np.linalg.norm(Vg - Vr) <= 1e-7 * np.linalg.norm(Vr), i


@pytest.mark.parametrize("kw", [dict(warm_start=0), dict(extrapolate=0),
                                dict(T_c=2, gamma_c=0.01, rearm_at_switch=0),
                                dict(rearm_at_switch=0), dict(step_rule=1),
                                dict(step_rule=1, rearm_at_switch=0)])
def test_fp64_option_variants(kw):
    """A-WMMSE, no extrapolation, fixed gamma_c, single adaptive window, the
    frozen step rule (with and without the re-armed window)."""
    b = synth.pack([random_instance(110, M=8, cell_users=[2, 2], N=2, d=2, P=[4.0, 6.0]),
                    random_instance(111, M=12, cell_users=[4], N=2, d=1, P=3.0)])
    # the frozen rule keeps a step from a smaller curvature in stage II and
    # oscillates there; rounding differences then grow geometrically, so those
    # variants are compared over a shorter run
    T = 16 if kw.get("step_rule") == 1 else 60
    okw = dict(iters=T)
    if "warm_start" in kw:
        okw["warm_start"] = False
    if "extrapolate" in kw:
        okw["extrapolate"] = False
    if "T_c" in kw:
        okw.update(Tc=kw["T_c"], gamma_c=kw["gamma_c"])
    if "rearm_at_switch" in kw:
        okw["rearm_at_switch"] = bool(kw["rearm_at_switch"])
    if "step_rule" in kw:
        okw["step_rule"] = "frozen"
    refs = oracle_runs(b, range(b.batch), **okw)
    fs = np.array([r["switch_iter"] if r["switch_iter"] > 0 else 0 for r in refs], np.int32)
    say("case: variants", kw)
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=T, **kw),
                      want_trace=True, force_switch=fs)
    for i, ref in enumerate(refs):
        np.testing.assert_allclose(res.trace[i], ref["trace"], rtol=1e-9, err_msg=str((kw, i)))


def test_fp64_eps2_early_stop():
    b = synth.pack([random_instance(120, M=6, cell_users=[3], N=2, d=2, P=3.0),
                    random_instance(121, M=10, cell_users=[2, 2], N=2, d=1, P=[2.0, 2.0])])
    refs = oracle_runs(b, range(b.batch), iters=300, eps2=1e-3)
    say("case: eps2 stop")
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=300, eps2=1e-3),
                      want_trace=True)
    for i, ref in enumerate(refs):
        assert res.iters[i] == ref["iters"], (i, res.iters[i], ref["iters"])
        assert res.iters[i] < 300
        assert res.wsr[i] == pytest.approx(ref["wsr"], rel=1e-9)
        n = ref["iters"]
        np.testing.assert_allclose(res.trace[i, :n + 1], ref["trace"][:n + 1], rtol=1e-9)
        assert np.all(np.isnan(res.trace[i, n + 1:]))


def test_zero_budget_and_zero_iterations():
    """P_c = 0 keeps that BS silent (status bit), T = 0 returns WSR(V0)."""
    a = random_instance(130, M=6, cell_users=[2, 2], N=2, d=2, P=[3.0, 0.0])
    a["V0"][1][:] = 0
    b = synth.pack([a, random_instance(131, M=6, cell_users=[3], N=2, d=2, P=3.0)])
    refs = oracle_runs(b, range(b.batch), iters=20)
    say("case: zero budget")
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=20), want_trace=True)
    assert res.status[0] == ammse.INST_ZERO_POWER and res.status[1] == 0
    for i, ref in enumerate(refs):
        np.testing.assert_allclose(res.trace[i], ref["trace"], rtol=1e-9)
    r0 = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=0), want_trace=True)
    assert np.all(r0.iters == 0)
    np.testing.assert_allclose(r0.wsr, [r["trace"][0] for r in refs], rtol=1e-12)
    np.testing.assert_array_equal(r0.V, b.V0)


def test_wsr_entry_point():
    b = _ragged_batch()
    rng = np.random.default_rng(7)
    V = b.V0 + 0.3 * (rng.standard_normal(b.V0.shape) + 1j * rng.standard_normal(b.V0.shape))
    ref = []
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        ref.append(O.wsr_bits(prob, O.split_v(prob, v_blocks(b, V, i))))
    say("case: wsr entry point")
    g64 = ammse.wsr(b, V, precision=ammse.PREC_FP64)
    np.testing.assert_allclose(g64, ref, rtol=1e-12)
    g32 = ammse.wsr(b, V, precision=ammse.PREC_FP32)
    np.testing.assert_allclose(g32, ref, rtol=2e-5)


# ---------------------------------------------------------------------------
# FP32: WSR-level parity on the workloads
# ---------------------------------------------------------------------------

def test_fp32_rayleigh_sweep_subset():
    """Eight instances of the benchmark sweep (two per SNR) in their own launch:
    the whole WSR trajectory within 1e-4 of the oracle."""
    b = synth.rayleigh_sweep(B_per_p=3)
    idx = [0, 1, 3, 4, 6, 7, 9, 10]
    sub = b.subset(idx)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: rayleigh sweep fp32 subset")
    res = ammse.solve(sub, opts, want_trace=True)
    assert np.all(res.status == 0)
    refs = oracle_runs(sub, range(sub.batch), iters=100)
    compare_traces(sub, res, refs, list(range(sub.batch)), opts, 1e-4)


def test_fp32_full_bench_batch_sampled():
    """The benchmarked launch (1024 instances, M=64, 16 users, N=d=4, all four
    SNRs, T=100) in one call: 32 instances (8 per SNR, stored FP64 oracle runs)
    to 1e-4 over the whole trajectory, properties on every instance."""
    b = synth.rayleigh_sweep(B_per_p=256)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: full 1024-instance fp32 launch")
    res = ammse.solve(b, opts, want_trace=True)
    assert np.all(res.status == 0)
    assert np.all(np.isfinite(res.wsr)) and np.all(res.wsr > 0)
    assert np.all(np.isfinite(res.trace))
    assert np.all((res.switch_iter >= 2) & (res.switch_iter <= 100))
    for i in range(b.batch):
        Vi = res.V[b.v_off[i]: b.v_off[i] + 64 * 64]
        assert np.vdot(Vi, Vi).real <= b.P[i] * (1 + 1e-5)
    g = golden("wmmse_ref_rayleigh_sweep4x256.json")["ammmse"]
    refs = [dict(trace=g["trace"][k], switch_iter=g["switch_iter"][k], wsr=g["wsr"][k])
            for k in range(len(g["index"]))]
    compare_traces(b, res, refs, g["index"], opts, 1e-4)
    same = [res.switch_iter[i] == r["switch_iter"] for i, r in zip(g["index"], refs)]
    say("switch agreement", sum(same), "of", len(same))


def test_fp64_hexcell_iterates():
    """Seven-cell instances with path loss (uneven users, M, N) in FP64: the
    whole 100-iteration WSR trajectory to 1e-9 and the precoders after 20
    iterations to 1e-10 of their norm."""
    b = synth.hexcell_batch(B=12)
    idx = [0, 3, 5, 8]
    sub = b.subset(idx)
    refs = oracle_runs(sub, range(sub.batch), iters=100)
    refs20 = oracle_runs(sub, range(sub.batch), iters=20)
    fs = np.array([r["switch_iter"] for r in refs], np.int32)
    say("case: hexcell fp64 T=100")
    res = ammse.solve(sub, ammse.Options(precision=ammse.PREC_FP64, max_iters=100),
                      want_trace=True, force_switch=fs)
    res20 = ammse.solve(sub, ammse.Options(precision=ammse.PREC_FP64, max_iters=20),
                        force_switch=fs)
    assert np.all(res.status == 0)
    for i, ref in enumerate(refs):
        np.testing.assert_allclose(res.trace[i], ref["trace"], rtol=1e-9)
        Vg = np.concatenate([x.ravel() for x in v_blocks(sub, res20.V, i)])
        Vr = np.concatenate([x.ravel() for x in
                             O.join_v(O.from_instance(sub.instance(i)), refs20[i]["V"])])
        assert np.linalg.norm(Vg - Vr) <= 1e-10 * np.linalg.norm(Vr)


def test_fp32_hexcell_small_batch():
    """FP32 on four seven-cell instances in their own launch: the whole WSR
    trajectory within 1e-4 of the oracle; finite and feasible precoders."""
    b = synth.hexcell_batch(B=12)
    idx = [0, 3, 5, 8]
    sub = b.subset(idx)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    refs = oracle_runs(sub, range(sub.batch), iters=100)
    say("case: hexcell fp32 T=100")
    res = ammse.solve(sub, opts, want_trace=True)
    assert np.all(res.status == 0)
    compare_traces(sub, res, refs, list(range(sub.batch)), opts, 1e-4)
    for i in range(sub.batch):
        assert np.all(np.isfinite(res.trace[i])) and res.wsr[i] > 0
        inst = sub.instance(i)
        for c, Vc in enumerate(v_blocks(sub, res.V, i)):
            assert np.vdot(Vc, Vc).real <= inst["P"][c] * (1 + 1e-5)


def test_fp32_hexcell_full_launch_sampled():
    """The seven-cell launch the benchmark times: all 4096 uneven instances in
    one persistent launch with the autotuned tile shapes.  32 stored oracle runs
    (16 per tile-shape class present) to 1e-4 over the whole trajectory, status,
    finiteness and feasibility on every instance."""
    b = synth.hexcell_batch(4096)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: hexcell 4096 fp32 launch (autotuned)")
    res = ammse.solve(b, opts, want_trace=True, autotune=True)
    assert np.all(res.status == 0)
    assert np.all(np.isfinite(res.wsr)) and np.all(res.wsr > 0)
    for i in range(0, b.batch, 97):
        inst = b.instance(i)
        for c, Vc in enumerate(v_blocks(b, res.V, i)):
            assert np.vdot(Vc, Vc).real <= inst["P"][c] * (1 + 1e-5)
    g = golden("oracle_ref_hexcell7_b4096.json")["ammmse"]
    assert set(g["shape_class"]) == {0, 1}
    refs = [dict(trace=g["trace"][k], switch_iter=g["switch_iter"][k], wsr=g["wsr"][k])
            for k in range(len(g["index"]))]
    compare_traces(b, res, refs, g["index"], opts, 1e-4)


def test_fp32_large_instance_sample():
    b = synth.rayleigh_large(B=2)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: M=256 U=64 fp32")
    res = ammse.solve(b, opts)
    assert np.all(res.status == 0)
    refs = oracle_runs(b, [0, 1], iters=100)
    compare_wsr(b, res, refs, [0, 1], opts, 1e-4)


# ---------------------------------------------------------------------------
# LDS-resident MFMA kernel (selected automatically for its shapes)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("U,N,d", [(16, 4, 4), (32, 2, 2), (64, 1, 1)])
def test_fp32_lds_kernel_shapes_vs_oracle(U, N, d):
    """Single-cell M = 64, U*N = U*d = 64 for N = 4, 2, 1 (the shapes the
    LDS-resident kernel serves), all four SNRs: the whole WSR trajectory
    within 1e-4 of the oracle."""
    insts = [random_instance(200 + k, M=64, cell_users=[U], N=N, d=d, P=10.0 ** k,
                             alpha_range=(0.5, 1.5)) for k in range(4)]
    b = synth.pack(insts)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: lds kernel", U, N, d)
    res = ammse.solve(b, opts, want_trace=True)
    assert np.all(res.status == 0)
    refs = oracle_runs(b, range(b.batch), iters=100)
    compare_traces(b, res, refs, list(range(b.batch)), opts, 1e-4)


def test_lds_kernel_matches_general_kernel():
    """Both FP32 kernels on the same 64 instances (16 per SNR): identical stage
    decisions for nearly all and, where they agree, whole WSR trajectories
    within 2e-4 of each other (each within 1e-4 of the oracle)."""
    b = synth.rayleigh_sweep(B_per_p=16)
    say("case: lds vs general")
    fast = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP32, max_iters=100),
                       want_trace=True)
    gen = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP32, max_iters=100,
                                       path=ammse.PATH_GENERAL), want_trace=True)
    same = fast.switch_iter == gen.switch_iter
    assert same.mean() >= 0.9
    np.testing.assert_allclose(fast.trace[same], gen.trace[same], rtol=2e-4)
    np.testing.assert_allclose(fast.wsr[same], gen.wsr[same], rtol=2e-4)


def test_lds_kernel_without_trace_matches_traced_run():
    """Without a trace and eps2 = 0 the LDS kernel skips the per-iteration WSR
    reduction in stage II; the iterates do not depend on it, so the precoders,
    WSR, switch iteration and status equal those of the traced run."""
    b = synth.rayleigh_sweep(B_per_p=8)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100)
    say("case: lds kernel with / without trace")
    a = ammse.solve(b, opts, want_trace=True)
    c = ammse.solve(b, opts, want_trace=False)
    np.testing.assert_array_equal(c.switch_iter, a.switch_iter)
    np.testing.assert_array_equal(c.status, a.status)
    np.testing.assert_array_equal(c.V, a.V)
    np.testing.assert_array_equal(c.wsr, a.wsr)


@pytest.mark.parametrize("eps2", [0.0, 1e-4])
def test_general_q_path_rebuilds_the_returned_precoder(eps2):
    """Single-cell instances with U N <= M on the general kernel in float (one
    product with Q per iteration, V carried as c V^0 + H^H S X and rebuilt at
    the end, also after an eps2 stop): the reported WSR is the WSR of the
    returned precoders (ammse_wsr) and every precoder meets its budget."""
    b = synth.rayleigh_large(6, seed=24777)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=100, eps2=eps2,
                         path=ammse.PATH_GENERAL)
    say("case: general Q path rebuild, eps2", eps2)
    res = ammse.solve(b, opts)
    assert np.all(res.status == 0)
    if eps2 > 0:
        assert np.any(res.iters < 100)
    w = ammse.wsr(b, res.V, precision=ammse.PREC_FP32)
    np.testing.assert_allclose(res.wsr, w, rtol=1e-6)
    n = int(b.M[0]) * int(b.U[0]) * int(b.d[0])
    for i in range(b.batch):
        Vi = res.V[b.v_off[i]: b.v_off[i] + n]
        assert np.vdot(Vi, Vi).real <= b.P[i] * (1 + 1e-5)


@pytest.mark.parametrize("variant", ["eps2", "no_extrapolation", "no_warm_start", "forced_switch"])
def test_lds_kernel_option_variants(variant):
    """The LDS-resident kernel under the option variants (eps2 stop, omega = 0,
    A-WMMSE without warm start, a forced stage switch): the reported WSR is the
    WSR of the returned precoders (ammse_wsr), every precoder meets its budget,
    and at every SNR the WSR trajectory follows the oracle run with the same
    options to 1e-4 (up to the stop iteration with eps2)."""
    okw, gkw = {"eps2": (dict(eps2=1e-4), dict(eps2=1e-4)),
                "no_extrapolation": (dict(extrapolate=False), dict(extrapolate=0)),
                "no_warm_start": (dict(warm_start=False), dict(warm_start=0)),
                "forced_switch": (dict(force_switch_iter=5), dict(force_switch_iter=5))}[variant]
    T = 60
    b = synth.rayleigh_sweep(B_per_p=2)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=T, **gkw)
    say("case: lds kernel variant", variant)
    res = ammse.solve(b, opts, want_trace=True)
    assert np.all(res.status == 0)
    if variant == "forced_switch":
        assert np.all(res.switch_iter == 5)
    if variant == "eps2":
        assert np.any(res.iters < T)
    w = ammse.wsr(b, res.V, precision=ammse.PREC_FP32)
    np.testing.assert_allclose(res.wsr, w, rtol=1e-6)
    n = 64 * 16 * 4
    for i in range(b.batch):
        Vi = res.V[b.v_off[i]: b.v_off[i] + n]
        assert np.vdot(Vi, Vi).real <= b.P[i] * (1 + 1e-5)
    refs = oracle_runs(b, range(b.batch), iters=T, **okw)
    for i, ref in enumerate(refs):
        tr = res.trace[i]
        if res.switch_iter[i] != ref["switch_iter"]:
            r2 = ammse.solve(b.subset([i]), opts, want_trace=True,
                             force_switch=np.array([ref["switch_iter"]], np.int32))
            tr = r2.trace[0]
        if variant == "eps2":
            assert abs(int(res.iters[i]) - ref["iters"]) <= 2, (i, res.iters[i], ref["iters"])
            m = min(int(res.iters[i]), ref["iters"]) + 1
        else:
            m = T + 1
        np.testing.assert_allclose(tr[:m], ref["trace"][:m], rtol=1e-4, err_msg=str(i))


def test_lanczos_order_beyond_the_lds_vectors():
    """Single cell with U N = 520 <= M = 528, FP64: the step size runs Lanczos
    of order 520, above the 512 whose vectors the general kernel keeps in LDS,
    so its vectors stay in the workspace; the WSR trajectory over 20 iterations
    (the adaptive step sizes of both windows, then the stage-II bound, whose
    Lanczos on the antenna side has order 528) matches the oracle to 1e-9."""
    b = synth.pack([random_instance(321, M=528, cell_users=[130], N=4, d=1, P=100.0)])
    opts = ammse.Options(precision=ammse.PREC_FP64, max_iters=20, path=ammse.PATH_GENERAL)
    say("case: Lanczos order 520, FP64")
    res = ammse.solve(b, opts, want_trace=True)
    assert res.status[0] == 0
    ref = oracle_runs(b, [0], iters=20)[0]
    tr = res.trace[0]
    if res.switch_iter[0] != ref["switch_iter"]:
        tr = ammse.solve(b, opts, want_trace=True,
                         force_switch=np.array([ref["switch_iter"]], np.int32)).trace[0]
    np.testing.assert_allclose(tr, ref["trace"], rtol=1e-9)


@pytest.mark.parametrize("cells,M,N,d", [([10, 12, 8], 64, 2, 2), ([30, 40, 20], 64, 1, 1),
                                         ([30, 40, 20], 48, 1, 1), ([48, 48], 128, 2, 2),
                                         ([50, 50], 256, 2, 2)])
def test_fp32_gram_step_size_orders(cells, M, N, d):
    """FP32 multi-cell instances whose step size comes from the Lanczos
    iteration on a Gram matrix, R_c R_c^H ((U d) x (U d)) or R_c^H R_c (M x M),
    whichever is smaller: stream side of order 60, antenna side of order 64,
    48 (ragged: not a multiple of the 8-column chunks) and 128, all one wave
    per BS, and stream side of order 200 (above the 192 the per-wave
    iteration holds), the block-wide one; the WSR trajectory over 30
    iterations matches the oracle's to the FP32 bound."""
    b = synth.pack([random_instance(700 + M + 7 * N, M=M, cell_users=cells, N=N, d=d, P=10.0)])
    ud, un = d * sum(cells), N * sum(cells)
    ng = min(ud, M)
    assert ng * ng < 2 * un * M   # the Gram form is the cheaper step-size operator
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=30, path=ammse.PATH_GENERAL)
    say("case: gram step size", cells, M, "order", ng)
    res = ammse.solve(b, opts, want_trace=True)
    assert res.status[0] == 0
    refs = oracle_runs(b, [0], iters=30)
    compare_traces(b, res, refs, [0], opts, 1e-4)


@pytest.mark.parametrize("cells,M,N,d", [([3, 5], 16, 1, 1), ([4, 6, 2], 32, 2, 2),
                                         ([5, 3], 48, 4, 2), ([7, 9, 4], 24, 2, 1),
                                         ([12], 16, 2, 2)])
def test_fp32_small_antenna_products(cells, M, N, d):
    """FP32 instances whose channel products have few rows or columns: the
    gradient products H^H Z and the antenna-side Gram matrices with M <= 32
    output rows (16- and 32-row tiles, the k-chunks split over wave groups),
    M = 48 (a 64-row tile with a ragged row block), M = 24 (a ragged k-chunk in
    the channel products), channel products with U N <= 64 rows, a single
    cell with U N > M (two-product form); WSR trajectories over 40 iterations
    against the oracle at the FP32 bound."""
    b = synth.pack([random_instance(800 + M + 11 * N + len(cells), M=M, cell_users=cells, N=N,
                                    d=d, P=10.0, alpha_range=(0.5, 1.5))])
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=40, path=ammse.PATH_GENERAL)
    say("case: small-antenna products", cells, M, N, d)
    res = ammse.solve(b, opts, want_trace=True)
    assert res.status[0] == 0
    refs = oracle_runs(b, [0], iters=40)
    compare_traces(b, res, refs, [0], opts, 1e-4)


@pytest.mark.parametrize("U,M,N,d", [(9, 20, 1, 1), (7, 30, 2, 2), (5, 17, 3, 2), (6, 40, 4, 3),
                                     (40, 130, 3, 2)])
def test_q_path_every_receive_dimension(U, M, N, d):
    """Single-cell instances on the Q path (U N <= M) for every N: the step
    size's K = C^H Q C (formed per N, entries below the diagonal from their
    mirrors) and its Lanczos products in column chunks with ragged ends (U N
    not a multiple of the chunk; U N = 120 > 64 spans several wave rows).
    FP64 trajectories to 1e-9 and FP32 to the FP32 bound, against the oracle."""
    b = synth.pack([random_instance(900 + 10 * N + U, M=M, cell_users=[U], N=N, d=d, P=20.0,
                                    alpha_range=(0.5, 1.5))])
    T = 40
    refs = oracle_runs(b, [0], iters=T)
    say("case: q path", U, M, N, d)
    res = ammse.solve(b, ammse.Options(precision=ammse.PREC_FP64, max_iters=T), want_trace=True,
                      force_switch=np.array([refs[0]["switch_iter"]], np.int32))
    assert res.status[0] == 0
    np.testing.assert_allclose(res.trace[0], refs[0]["trace"], rtol=1e-9)
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=T, path=ammse.PATH_GENERAL)
    res = ammse.solve(b, opts, want_trace=True)
    assert res.status[0] == 0
    compare_traces(b, res, refs, [0], opts, 1e-4)
