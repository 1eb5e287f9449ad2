"""Unrolled A-MMMSE (forward + hand-written adjoint kernels) against the FP64
oracle of the unrolled solver (torch autograd on the paper's steps, pinned by
finite differences in tests/test_unrolled_oracle.py).

Bars: FP64 forward WSR and trace within 1e-10 of the oracle, with the stage
switch the oracle's own eps1 rule picks; FP64 gradients (step sizes and
channel) within 1e-8 relative in norm, at small shapes and at the M=64,
16-user, N=d=4, P=20 dB, T=20 shape with the paper's step schedule; there
FP32 gradients within 2e-3 of the oracle's (relative, in norm); gradients
independent of the checkpoint interval; the FP64 kernel's step-size gradient
within 1e-5 of central differences with h = 1e-3 gamma_t, and its channel
gradient along a random direction within 1e-5 of central differences with
h = 1e-3; a step schedule shared by the batch receives the sum of the
per-instance gradients.
"""
import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth
import oracle as O
from instances import random_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def say(*a):
    print(*a, flush=True)


def _steps(b, T, lo=0.8, hi=1.2):
    """Per-instance step schedules around the paper's first adaptive step."""
    out = np.zeros((b.batch, T))
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        V0 = O.split_v(prob, inst["V0"])
        Uu = O.mmse_receivers(prob, V0)
        Wu = np.stack([np.eye(prob.d)] * prob.U)
        g0 = O.step_sizes(O.transmit_hessians(prob, Uu, Wu))[0]
        out[i] = g0 * np.linspace(lo, hi, T)
    return out


def _run(b, gam, prec, K, dwsr=None, force=None):
    import torch
    T = gam.shape[1]
    opts = ammse.Options(precision=prec, max_iters=T)
    db = ammse.to_device(b, prec)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    ws_b, ck_b = plan.unrolled_sizes(K)
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    ck = torch.empty(ck_b, dtype=torch.uint8, device="cuda")
    B = b.batch
    V = db.V0.clone()
    g = torch.from_numpy(np.ascontiguousarray(gam)).cuda()
    wsr = torch.empty(B, dtype=torch.float64, device="cuda")
    sw = torch.empty(B, dtype=torch.int32, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    tr = torch.empty((B, T + 1), dtype=torch.float64, device="cuda")
    fs = None if force is None else torch.from_numpy(np.asarray(force, np.int32)).cuda()
    plan.unrolled_forward(db.H, db.sigma2, db.alpha, db.P, V, g, K, wsr, sw, ck, ws, status=st,
                          trace=tr, force_switch=fs)
    dw = torch.ones(B, dtype=torch.float64, device="cuda") if dwsr is None else \
        torch.from_numpy(np.asarray(dwsr, float)).cuda()
    dH = torch.empty_like(db.H)
    dg = torch.empty_like(g)
    plan.unrolled_backward(db.H, db.sigma2, db.alpha, db.P, g, K, sw, ck, dw, dH, dg, ws)
    torch.cuda.synchronize()
    out = dict(wsr=wsr.cpu().numpy(), sw=sw.cpu().numpy(), st=st.cpu().numpy(),
               trace=tr.cpu().numpy(), dH=dH.cpu().numpy().astype(np.complex128),
               dg=dg.cpu().numpy(), V=V.cpu().numpy().astype(np.complex128))
    plan.close()
    return out


def _small():
    insts = [random_instance(41, M=6, cell_users=[3], N=2, d=2, P=10.0, alpha_range=(0.5, 1.5)),
             random_instance(42, M=10, cell_users=[4], N=3, d=2, P=5.0, sigma2=0.5,
                             alpha_range=(0.5, 1.5)),
             random_instance(43, M=5, cell_users=[2], N=1, d=1, P=20.0)]
    return synth.pack(insts, name="unroll_small")


def _h_block(b, arr, i):
    inst = b.instance(i)
    n = inst["U"] * inst["N"] * inst["M"]
    return arr[b.h_off[i]: b.h_off[i] + n].reshape(inst["U"], inst["N"], inst["M"])


def test_fp64_forward_and_gradients_match_oracle():
    b = _small()
    T = 8
    gam = _steps(b, T)
    res = _run(b, gam, ammse.PREC_FP64, K=3)
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        V0 = O.split_v(prob, inst["V0"])
        sw = O_unrolled().switch_iter(prob.Hs[:, 0], prob.sigma2, prob.alpha, prob.P[0], V0,
                                      gam[i])
        assert (int(res["sw"][i]) if res["sw"][i] >= 1 else T + 1) == sw, (i, res["sw"][i], sw)
        w, gg, gH, VT, trace = O_unrolled().value_and_grad(prob.Hs[:, 0], prob.sigma2, prob.alpha,
                                                           prob.P[0], V0, gam[i], sw)
        say(f"instance {i}: switch {res['sw'][i]}, wsr gpu {res['wsr'][i]:.12f} oracle {w:.12f}")
        assert res["st"][i] == 0
        assert res["wsr"][i] == pytest.approx(w, rel=1e-10)
        np.testing.assert_allclose(res["trace"][i][:T], trace, rtol=1e-10)
        err_g = np.linalg.norm(res["dg"][i] - gg) / np.linalg.norm(gg)
        dHi = _h_block(b, res["dH"], i)
        err_h = np.linalg.norm(dHi - gH) / np.linalg.norm(gH)
        say(f"   dgamma rel err {err_g:.2e}, dH rel err {err_h:.2e}")
        assert err_g <= 1e-8 and err_h <= 1e-8


def O_unrolled():
    from oracle import unrolled
    return unrolled


def test_gradients_do_not_depend_on_the_checkpoint_interval():
    b = _small()
    T = 8
    gam = _steps(b, T)
    ref = _run(b, gam, ammse.PREC_FP64, K=T)
    for K in (1, 3):
        r = _run(b, gam, ammse.PREC_FP64, K=K)
        np.testing.assert_array_equal(r["wsr"], ref["wsr"])
        np.testing.assert_allclose(r["dg"], ref["dg"], rtol=1e-13, atol=0)
        np.testing.assert_allclose(r["dH"], ref["dH"], rtol=1e-13,
                                   atol=1e-13 * np.abs(ref["dH"]).max())


def test_upstream_weights_scale_the_gradients():
    b = _small()
    T = 6
    gam = _steps(b, T)
    a = _run(b, gam, ammse.PREC_FP64, K=2)
    w = np.array([2.0, -0.5, 0.0])
    c = _run(b, gam, ammse.PREC_FP64, K=2, dwsr=w)
    np.testing.assert_allclose(c["dg"], a["dg"] * w[:, None], rtol=1e-12, atol=1e-300)


def _unroll_batch(B=6):
    return synth.unrolled_batch(B)


def _paper_steps(b, T):
    """The paper's step schedule for each instance (adaptive steps for t <= T_c
    and again at the switch, then kept) and its switch iteration, from the
    FP64 oracle: the natural initialisation of learnable unrolled steps."""
    g = np.zeros((b.batch, T))
    sw = np.zeros(b.batch, np.int32)
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        r = O.ammmse(prob, O.split_v(prob, inst["V0"]), T)
        g[i] = np.asarray(r["gammas"])[:, 0]
        sw[i] = r["switch_iter"] if r["switch_iter"] >= 1 else T + 1
    return g, sw


def test_fp32_gradients_match_fp64_at_full_shape():
    b = _unroll_batch(6)
    T = 20
    gam, fs = _paper_steps(b, T)
    r64 = _run(b, gam, ammse.PREC_FP64, K=5, force=fs)
    r32 = _run(b, gam, ammse.PREC_FP32, K=5, force=fs)
    for i in range(b.batch):
        eg = np.linalg.norm(r32["dg"][i] - r64["dg"][i]) / np.linalg.norm(r64["dg"][i])
        eh = np.linalg.norm(_h_block(b, r32["dH"], i) - _h_block(b, r64["dH"], i)) / \
            np.linalg.norm(_h_block(b, r64["dH"], i))
        say(f"instance {i}: switch {fs[i]}, fp32 vs fp64: dgamma {eg:.2e}, dH {eh:.2e}, "
            f"wsr {abs(r32['wsr'][i] - r64['wsr'][i]) / r64['wsr'][i]:.2e}")
        assert eg <= 2e-3 and eh <= 2e-3


@pytest.mark.parametrize("prec,tol", [(ammse.PREC_FP64, 1e-8), (ammse.PREC_FP32, 2e-3)])
def test_gradients_match_oracle_at_full_shape(prec, tol):
    """Two instances of the M=64, 16-user, N=d=4, P=20 dB batch, T=20 with the
    paper's step schedule, checkpoints every 5: forward WSR, stage switch (the
    oracle's own eps1 decision), step-size and channel gradients against the
    oracle of the unrolled solver."""
    b = _unroll_batch(2)
    T = 20
    gam, _ = _paper_steps(b, T)
    res = _run(b, gam, prec, K=5)
    for i in range(b.batch):
        inst = b.instance(i)
        prob = O.from_instance(inst)
        V0 = O.split_v(prob, inst["V0"])
        H = prob.Hs[:, 0]
        sw = O_unrolled().switch_iter(H, prob.sigma2, prob.alpha, prob.P[0], V0, gam[i])
        gsw = int(res["sw"][i]) if res["sw"][i] >= 1 else T + 1
        r = res
        if gsw != sw:   # a borderline eps1 decision in float: follow the oracle's branch
            r = _run(b, gam, prec, K=5, force=np.array([sw] * b.batch, np.int32))
        w, gg, gH, _, _ = O_unrolled().value_and_grad(H, prob.sigma2, prob.alpha, prob.P[0], V0,
                                                      gam[i], sw)
        eg = np.linalg.norm(r["dg"][i] - gg) / np.linalg.norm(gg)
        eh = np.linalg.norm(_h_block(b, r["dH"], i) - gH) / np.linalg.norm(gH)
        ew = abs(r["wsr"][i] - w) / w
        say(f"instance {i} prec {prec}: switch gpu {gsw} oracle {sw}, wsr {ew:.2e}, "
            f"dgamma {eg:.2e}, dH {eh:.2e}")
        if prec == ammse.PREC_FP64:
            assert gsw == sw
        assert ew <= (1e-10 if prec == ammse.PREC_FP64 else 1e-4)
        assert eg <= tol and eh <= tol


def test_fp64_channel_gradient_matches_central_differences_at_full_shape():
    """d/dh WSR(H + h Delta) at h = 0 by central differences (h = 1e-3, Delta a
    random complex direction of unit norm per instance, stage switch held
    fixed) against Re <dH, Delta> from the adjoint, at the full shape."""
    b = _unroll_batch(2)
    T = 20
    gam, fs = _paper_steps(b, T)
    base = _run(b, gam, ammse.PREC_FP64, K=5, force=fs)
    rng = np.random.default_rng(77)
    Dl = rng.standard_normal(b.H.shape) + 1j * rng.standard_normal(b.H.shape)
    blocks = [slice(int(b.h_off[i]), int(b.h_off[i]) + int(b.U[i] * b.N[i] * b.M[i]))
              for i in range(b.batch)]
    for blk in blocks:
        Dl[blk] /= np.linalg.norm(Dl[blk])
    h = 1e-3

    def shifted(sign):
        bb = b.subset(range(b.batch))
        bb.H = b.H + sign * h * Dl
        return _run(bb, gam, ammse.PREC_FP64, K=5, force=fs)["wsr"]

    fd = (shifted(+1) - shifted(-1)) / (2 * h)
    adj = np.array([np.real(np.vdot(base["dH"][blk], Dl[blk])) for blk in blocks])
    say(f"channel direction: adjoint {adj}, central difference {fd}")
    np.testing.assert_allclose(adj, fd, rtol=1e-5)


def test_fp64_step_gradient_matches_central_differences():
    b = _unroll_batch(2)
    T = 20
    gam, fs = _paper_steps(b, T)
    base = _run(b, gam, ammse.PREC_FP64, K=5, force=fs)
    for t in (0, 7, 19):
        h = 1e-3 * gam[:, t]
        gp, gm = gam.copy(), gam.copy()
        gp[:, t] += h
        gm[:, t] -= h
        fp = _run(b, gp, ammse.PREC_FP64, K=5, force=fs)["wsr"]
        fm = _run(b, gm, ammse.PREC_FP64, K=5, force=fs)["wsr"]
        fd = (fp - fm) / (2 * h)
        say(f"t={t + 1}: adjoint {base['dg'][:, t]}, central difference {fd}")
        np.testing.assert_allclose(base["dg"][:, t], fd, rtol=1e-5,
                                   atol=1e-7 * np.abs(base["dg"]).max())


def test_autograd_function():
    import torch
    from paper_2510_20507_amd.unrolled import unrolled_wsr
    b = _small()
    T = 6
    gam = _steps(b, T)
    ref = _run(b, gam, ammse.PREC_FP64, K=2)
    opts = ammse.Options(precision=ammse.PREC_FP64, max_iters=T)
    db = ammse.to_device(b, ammse.PREC_FP64)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    g = torch.from_numpy(gam).cuda().requires_grad_(True)
    H = db.H.clone().requires_grad_(True)
    wsr, VT, sw, st = unrolled_wsr(plan, db, g, H=H, ckpt_every=2)
    wsr.sum().backward()
    np.testing.assert_allclose(g.grad.cpu().numpy(), ref["dg"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(H.grad.cpu().numpy(), ref["dH"], rtol=1e-14, atol=0)
    # a step schedule shared by the batch receives the sum over instances
    gs = torch.from_numpy(gam[0]).cuda().requires_grad_(True)
    wsr2, _, _, _ = unrolled_wsr(plan, db, gs, ckpt_every=2)
    wsr2.sum().backward()
    assert gs.grad.shape == (T,)
    shared = np.tile(gam[0], (b.batch, 1))
    per = _run(b, shared, ammse.PREC_FP64, K=2)
    np.testing.assert_allclose(gs.grad.cpu().numpy(), per["dg"].sum(axis=0), rtol=1e-13,
                               atol=1e-13 * np.abs(per["dg"]).max())
    plan.close()
