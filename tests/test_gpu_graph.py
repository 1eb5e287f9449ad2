"""The batched solve captured in a HIP graph (torch.cuda.CUDAGraph over the
C ABI launch on the capture stream) and replayed: every replay, with eager
work and synchronisations in between, reproduces the eager launch bit for
bit (the solve records one kernel node and no memory-set node)."""
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


@pytest.mark.parametrize("kind", ["lds", "general", "bf16", "uneven"])
def test_graph_replays_match_eager(kind):
    import torch
    if kind == "uneven":
        b = synth.hexcell_batch(64, seed=23111)
        opts = ammse.Options(precision=ammse.PREC_FP32, max_iters=40)
    else:
        b = synth.rayleigh_sweep(B_per_p=16)
        opts = ammse.Options(precision=ammse.PREC_BF16 if kind == "bf16" else ammse.PREC_FP32,
                             max_iters=60,
                             path=ammse.PATH_GENERAL if kind == "general" else ammse.PATH_AUTO)
    db = ammse.to_device(b, opts.precision)
    plan = ammse.Plan(db.table, db.cell_users, opts)
    if kind == "lds":
        assert plan.kernel == ammse.KERNEL_LDS_MFMA
    ws = plan.workspace()
    B = b.batch
    V = torch.empty_like(db.V0)
    wsr = torch.empty(B, dtype=torch.float64, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    V.copy_(db.V0)
    plan.solve(db.H, db.sigma2, db.alpha, db.P, V, wsr, None, None, st, workspace=ws)
    torch.cuda.synchronize()
    V_ref, w_ref = V.clone(), wsr.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            V.copy_(db.V0)
            plan.solve(db.H, db.sigma2, db.alpha, db.P, V, wsr, None, None, st, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    for k in range(3):
        V.zero_()
        wsr.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(V, V_ref), (kind, k)
        assert torch.equal(wsr, w_ref), (kind, k)
        assert int(st.max()) == 0
    plan.close()
