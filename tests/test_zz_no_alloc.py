"""The allocation-free loss (elb_mlp_loss_noalloc, partial sums in the library's static
device scratch) against elb_mlp_loss with a caller workspace (needs an MI355X).

Both run the same kernels on the same inputs, so the loss and its gradient must agree bit
for bit.  Two calls in a row, the second with a smaller batch (fewer partial sums than the
first left in the scratch), check that nothing carries over between calls."""
import numpy as np
import pytest

from helpers import say

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _case(batch, q_out, seed, with_index):
    import torch
    import paper_2211_16933_amd as elb
    from paper_2211_16933_amd import learned
    rng = np.random.default_rng(seed)
    rows = batch + 11
    y = _dev(rng.normal(size=batch * 16).astype(np.float32))
    t = _dev(rng.normal(size=(rows, q_out)).astype(np.float32))
    norm = _dev(learned.make_norm(np.zeros(12), np.ones(12), rng.uniform(-0.2, 0.2, q_out),
                                  rng.uniform(0.5, 2.0, q_out), -np.full(12, 50.0),
                                  np.full(12, 50.0)))
    index = _dev(rng.permutation(rows)[:batch].astype(np.int32)) if with_index else None
    ws = torch.empty(elb.mlp_workspace_bytes(batch), dtype=torch.uint8, device="cuda:0")
    dy_ref = torch.full((batch * 16,), np.nan, dtype=torch.float32, device="cuda:0")
    dy = torch.full_like(dy_ref, np.nan)
    loss_ref = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    loss = torch.full_like(loss_ref, np.nan)
    say(f"case no-alloc loss batch={batch} q_out={q_out} index={with_index}")
    elb.mlp_loss(y, t, index, norm, batch, q_out, dy_ref, loss_ref, ws)
    elb.mlp_loss_noalloc(y, t, index, norm, batch, q_out, dy, loss)
    torch.cuda.synchronize()
    lr, ln = float(loss_ref.item()), float(loss.item())
    say(f"  loss with workspace {lr:.17g}, without {ln:.17g}")
    assert np.isfinite(lr) and lr > 0
    assert ln == lr
    assert torch.equal(dy, dy_ref)


def test_noalloc_loss_matches_workspace_loss_twice():
    # 20000 rows: the grid is capped at 256 blocks; then 300 rows: 19 blocks, so the
    # scratch still holds 237 stale partial sums of the first call
    _case(20000, 12, seed=1, with_index=True)
    _case(300, 8, seed=2, with_index=False)


def test_noalloc_loss_rejects_bad_sizes():
    import torch
    import paper_2211_16933_amd as elb
    y = torch.zeros(16, dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for batch, q_out in ((0, 8), ((1 << 24) + 1, 8), (1, 17)):
        with pytest.raises(elb.ElbError) as e:
            elb.mlp_loss_noalloc(y, y, None, y, batch, q_out, y, loss)
        assert e.value.code == elb.ELB_EINVAL
        say("  rejected:", e.value)
