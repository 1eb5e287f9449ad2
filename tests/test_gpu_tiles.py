"""Output tile shapes of the general kernel's MFMA channel products and the
autotuner that picks one per shape class.  Every tile shape computes each
product entry with the same k-order of MFMA accumulations, so forcing a
shape must not change the solve beyond float rounding; the autotuner only
reads V and leaves later solves unchanged in the same sense."""
import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def say(*a):
    print(*a, flush=True)


def _run(b, opts):
    res = ammse.solve(b, opts, want_trace=True)
    assert np.all(res.status == 0)
    return res


@pytest.mark.parametrize("prec", [ammse.PREC_FP32, ammse.PREC_BF16])
@pytest.mark.parametrize("kind", ["hexcell", "wide"])
def test_forced_tile_shapes_agree(kind, prec):
    """Uneven seven-cell batch (narrow per-cell blocks, classes 0 and 1) and
    64-user M = 256 instances (class 2): tile shapes 0, 1, 2 forced for every
    product give the same WSR trajectories and precoders."""
    b = synth.hexcell_batch(24, seed=23411) if kind == "hexcell" else synth.rayleigh_large(4)
    say("case: tiles", kind, prec)
    base = ammse.Options(precision=prec, max_iters=30, path=ammse.PATH_GENERAL)
    ref = _run(b, base)
    for tile in (1, 2, 3):
        o = ammse.Options(precision=prec, max_iters=30, path=ammse.PATH_GENERAL, tile=tile)
        res = _run(b, o)
        np.testing.assert_array_equal(res.switch_iter, ref.switch_iter)
        np.testing.assert_allclose(res.trace, ref.trace, rtol=1e-5)
        np.testing.assert_allclose(res.V, ref.V, rtol=0, atol=1e-4 * np.abs(ref.V).max())


def test_autotune_picks_per_class_and_keeps_results():
    import torch
    b = synth.pack([synth.hexcell_batch(24, seed=23412).instance(i) for i in range(24)] +
                   [synth.rayleigh_large(4).instance(i) for i in range(4)])
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=30, path=ammse.PATH_GENERAL)
    say("case: autotune")
    db = ammse.to_device(b, opts.precision)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    ws = plan.workspace()
    B = b.batch
    V = db.V0.clone()
    wsr0 = torch.empty(B, dtype=torch.float64, device="cuda")
    plan.solve(db.H, db.sigma2, db.alpha, db.P, V, wsr0, workspace=ws)
    V0c = db.V0.clone()
    choice = plan.autotune(db.H, db.sigma2, db.alpha, db.P, db.V0, workspace=ws)
    torch.cuda.synchronize()
    say("choice", choice)
    assert torch.equal(db.V0, V0c)                      # V is only read
    assert choice[2] in (0, 1, 2)                       # the M = 256 instances
    assert any(c in (0, 1, 2) for c in choice[:2])      # the seven-cell instances
    V2 = db.V0.clone()
    wsr1 = torch.empty(B, dtype=torch.float64, device="cuda")
    plan.solve(db.H, db.sigma2, db.alpha, db.P, V2, wsr1, workspace=ws)
    torch.cuda.synchronize()
    np.testing.assert_allclose(wsr1.cpu().numpy(), wsr0.cpu().numpy(), rtol=1e-5)
    plan.close()


@pytest.mark.parametrize("kind", ["lds", "fp64"])
def test_autotune_without_tile_choices(kind):
    import torch
    if kind == "lds":
        b = synth.rayleigh_sweep(B_per_p=2)
        opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=10)
    else:
        b = synth.hexcell_batch(4, seed=23413)
        opts = ammse.Options(precision=ammse.PREC_FP64, max_iters=10)
    db = ammse.to_device(b, opts.precision)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    assert plan.autotune(db.H, db.sigma2, db.alpha, db.P, db.V0) == [-1, -1, -1]
    plan.close()
