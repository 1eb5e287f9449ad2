"""Failure injection from the host: inputs that break an instance's numerics
must end that instance with the documented status bits and leave the other
instances of the launch untouched; nothing aborts and every call returns.

Every loop of the kernels is bounded independently of the data (Lanczos steps
by the Krylov dimension, the multisection rounds by a fixed count, the dual
search of the exact V step by 100 probes), so non-finite data cannot keep a
workgroup running.

Cases: NaN and Inf entries in H, a zero noise power (both make the
covariance factorisation or the WSR non-finite), an all-zero user channel
(valid: that user gets rate 0, the oracle's trajectory is followed), and
V^0 = 0 (valid: the gradient vanishes, V stays 0, WSR 0 and the zero-power
bit), in FP64 and FP32, on the general kernel and (float, 64-antenna shape)
on the LDS-resident one.
"""
import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth
import oracle as O
from instances import random_instance

pytestmark = pytest.mark.gpu

FAIL = ammse.INST_NONFINITE | ammse.INST_CHOLESKY


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def say(*a):
    print(*a, flush=True)


def _poison(inst, kind):
    inst = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in inst.items()}
    inst["H"] = [h.copy() for h in inst["H"]]
    inst["V0"] = [v.copy() for v in inst["V0"]]
    if kind == "nan_h":
        inst["H"][0][1, 3] = np.nan
    elif kind == "inf_h":
        inst["H"][-1][0, 0] = np.inf + 1j
    elif kind == "zero_sigma2":
        inst["sigma2"][0] = 0.0
    elif kind == "zero_user":
        for h in inst["H"]:
            h[0:inst["N"], :] = 0.0            # user 0 hears nothing from any BS
    elif kind == "zero_v0":
        for v in inst["V0"]:
            v[:] = 0.0
    return inst


SHAPES = {
    "general": lambda s: random_instance(s, M=12, cell_users=[3, 2], N=2, d=2, P=[5.0, 8.0],
                                         alpha_range=(0.5, 1.5)),
    "lds": lambda s: random_instance(s, M=64, cell_users=[16], N=4, d=4, P=100.0,
                                     alpha_range=(0.5, 1.5)),
}


@pytest.mark.parametrize("shape", ["general", "lds"])
@pytest.mark.parametrize("prec", [ammse.PREC_FP64, ammse.PREC_FP32])
@pytest.mark.parametrize("kind", ["nan_h", "inf_h", "zero_sigma2"])
def test_nonfinite_inputs_flag_the_instance_only(shape, prec, kind):
    good = [SHAPES[shape](900 + k) for k in range(3)]
    bad = _poison(SHAPES[shape](950), kind)
    b = synth.pack([good[0], bad, good[1], good[2]])
    ref = synth.pack(good)
    opts = ammse.Options(precision=prec, max_iters=30)
    say("case: failure", shape, prec, kind)
    res = ammse.solve(b, opts, want_trace=True)
    clean = ammse.solve(ref, opts, want_trace=True)
    assert res.status[1] & FAIL, res.status
    assert res.iters[1] < 30
    keep = [0, 2, 3]
    np.testing.assert_array_equal(res.status[keep], 0)
    np.testing.assert_array_equal(res.wsr[keep], clean.wsr)
    np.testing.assert_array_equal(res.trace[keep], clean.trace)
    nv = ref.V0.size // 3                       # the good instances share one shape
    for k, i in enumerate(keep):
        np.testing.assert_array_equal(res.V[b.v_off[i]: b.v_off[i] + nv],
                                      clean.V[ref.v_off[k]: ref.v_off[k] + nv])


@pytest.mark.parametrize("shape", ["general", "lds"])
def test_all_zero_user_channel_follows_the_oracle(shape):
    """A user with H_{u,j} = 0 for every BS is valid input: its rate is 0 and
    the iteration is the oracle's (FP64 trajectory 1e-9 on the general kernel;
    FP32 trajectory 1e-4 on the LDS-resident one)."""
    inst = _poison(SHAPES[shape](960), "zero_user")
    b = synth.pack([inst])
    prec = ammse.PREC_FP64 if shape == "general" else ammse.PREC_FP32
    tol = 1e-9 if shape == "general" else 1e-4
    T = 40
    prob = O.from_instance(inst)
    r = O.ammmse(prob, O.split_v(prob, inst["V0"]), T)
    say("case: zero user channel", shape)
    res = ammse.solve(b, ammse.Options(precision=prec, max_iters=T), want_trace=True,
                      force_switch=np.array([r["switch_iter"]], np.int32))
    assert res.status[0] == 0
    np.testing.assert_allclose(res.trace[0], r["trace"], rtol=tol)
    assert O.user_rates(prob, r["V"])[0] == 0.0


@pytest.mark.parametrize("shape", ["general", "lds"])
@pytest.mark.parametrize("prec", [ammse.PREC_FP64, ammse.PREC_FP32])
def test_zero_initial_precoder(shape, prec):
    """V^0 = 0: the receivers vanish, the gradient is 0, so V stays 0; WSR 0
    at every iteration, the zero-power bit set, as in the oracle."""
    inst = _poison(SHAPES[shape](970), "zero_v0")
    b = synth.pack([inst, SHAPES[shape](971)])
    T = 20
    prob = O.from_instance(inst)
    r = O.ammmse(prob, O.split_v(prob, inst["V0"]), T)
    assert np.all(r["trace"] == 0.0) and np.all(r["V"] == 0)
    say("case: zero V0", shape, prec)
    res = ammse.solve(b, ammse.Options(precision=prec, max_iters=T), want_trace=True)
    assert res.status[0] == ammse.INST_ZERO_POWER and res.status[1] == 0
    assert res.iters[0] == T and res.switch_iter[0] == r["switch_iter"]
    np.testing.assert_array_equal(res.trace[0], 0.0)
    np.testing.assert_array_equal(res.V[:int(b.v_off[1])], 0.0)
