"""The allocation-free solve (ammse_solve_noalloc) against ammse_solve.

Both run the same kernels; only the workspace differs (the library's static
device array instead of a caller buffer), so the results must be identical
bit for bit.  Two calls in a row, the second on a smaller plan, check that
nothing from the first call's contents of the shared array leaks into the
second; a plan whose workspace exceeds the array is refused.
"""
import ctypes

import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth
from instances import random_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ammse.lib()


def _run(batch, opts, noalloc):
    import torch
    db = ammse.to_device(batch, opts.precision)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    B = batch.batch
    V = db.V0.clone()
    out = dict(wsr=torch.full((B,), -1.0, dtype=torch.float64, device="cuda"),
               iters=torch.full((B,), -1, dtype=torch.int32, device="cuda"),
               sw=torch.full((B,), -1, dtype=torch.int32, device="cuda"),
               st=torch.full((B,), -1, dtype=torch.int32, device="cuda"),
               tr=torch.empty((B, opts.max_iters + 1), dtype=torch.float64, device="cuda"))
    args = (db.H, db.sigma2, db.alpha, db.P, V, out["wsr"], out["iters"], out["sw"], out["st"],
            out["tr"])
    if noalloc:
        assert plan.workspace_bytes <= ammse.SCRATCH_BYTES
        plan.solve_noalloc(*args)
    else:
        plan.solve(*args)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["V"] = V.cpu().numpy()
    plan.close()
    return res


def _same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _ragged(seed0, n):
    shapes = [dict(M=12, cell_users=[3, 2], N=2, d=2, P=[5.0, 8.0]),
              dict(M=70, cell_users=[5], N=1, d=1, P=10.0),
              dict(M=16, cell_users=[3, 3], N=4, d=4, P=[5.0, 5.0], sigma2=0.2),
              dict(M=66, cell_users=[20], N=4, d=3, P=30.0)]
    return synth.pack([random_instance(seed0 + k, alpha_range=(0.5, 1.5), **shapes[k % 4])
                       for k in range(n)])


@pytest.mark.parametrize("prec", [ammse.PREC_FP64, ammse.PREC_FP32])
def test_noalloc_matches_solve_on_two_calls(prec):
    """General kernel (its state lives in the workspace): 8 ragged instances,
    then 3 others; each call equals ammse_solve on the same inputs."""
    opts = ammse.Options(precision=prec, max_iters=40)
    for batch in (_ragged(1300, 8), _ragged(1400, 3)):
        print("case: noalloc", prec, batch.batch, flush=True)
        _same(_run(batch, opts, True), _run(batch, opts, False))


def test_noalloc_lds_kernel_and_seven_cell():
    """The LDS-resident kernel (64-antenna batch) and then a smaller seven-cell
    batch on the general kernel, in float, through the allocation-free call."""
    opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=60)
    for batch in (synth.rayleigh_sweep(B_per_p=8), synth.hexcell_batch(B=6)):
        print("case: noalloc fp32", batch.name, flush=True)
        _same(_run(batch, opts, True), _run(batch, opts, False))


def test_noalloc_refuses_a_plan_beyond_the_array():
    """A plan whose workspace exceeds AMMSE_SCRATCH_BYTES is refused
    (AMMSE_ERR_WORKSPACE) before anything is enqueued."""
    import torch
    b = synth.rayleigh_large(B=96)
    opts = ammse.Options(precision=ammse.PREC_FP64, max_iters=5)
    db = ammse.to_device(b, opts.precision)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    assert plan.workspace_bytes > ammse.SCRATCH_BYTES
    V = db.V0.clone()
    wsr = torch.full((b.batch,), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(ammse.AmmseError) as e:
        plan.solve_noalloc(db.H, db.sigma2, db.alpha, db.P, V, wsr)
    assert e.value.code == 4
    torch.cuda.synchronize()
    assert torch.equal(V, db.V0) and bool((wsr == -1.0).all())
    plan.close()
