"""The allocation-free loss/gradient entry point (we_mlp_loss_grad_noalloc)
against the allocating one (we_mlp_loss_grad), through the C ABI.

Both run the same forward/backward and gradient kernels on the same inputs,
so the loss and every gradient entry must be equal bit for bit.  Two calls in
a row, the second with a smaller batch and fewer inputs, check that the
shared fixed scratch carries nothing from one call into the next; a size
beyond the scratch must be refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _we():
    from paper_1303_5986_amd import we
    return we


def _case(rng, we, n_in, batch):
    n_p = we.n_params(n_in)
    params = (rng.standard_normal(n_p) * 0.3).astype(np.float32)
    feat = np.concatenate([rng.uniform(0.0, 4.0, n_in), 1.0 / rng.uniform(0.5, 2.0, n_in)]).astype(np.float32)
    x = rng.integers(0, 800, (batch, n_in)).astype(np.int32)
    y = rng.uniform(0.0, 1.0, batch).astype(np.float32)
    return params, feat, x, y


def test_noalloc_loss_grad_equals_allocating_entry_point():
    import torch
    we = _we()
    rng = np.random.default_rng(2024)
    dev = torch.device("cuda:0")
    for n_in, batch in ((8, 4096), (5, 300)):
        print(f"case: noalloc loss/grad n_in={n_in} batch={batch}", flush=True)
        params, feat, x, y = _case(rng, we, n_in, batch)
        loss0, g0 = we.mlp_loss_grad(n_in, params, feat, x, y)
        tp, tf, tx, ty = (torch.from_numpy(a).to(dev) for a in (params, feat, x, y))
        tl = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        tg = torch.full((len(g0),), float("nan"), dtype=torch.float32, device=dev)
        we.mlp_loss_grad_noalloc(n_in, tp, tf, tx, ty, tl, tg)
        torch.cuda.synchronize()
        loss1 = tl.cpu().numpy()
        g1 = tg.cpu().numpy()
        assert loss1.view(np.uint32)[0] == np.float32(loss0).view(np.uint32), (loss1[0], loss0)
        assert np.array_equal(g1.view(np.uint32), g0.view(np.uint32))
        assert np.isfinite(loss1[0]) and loss1[0] > 0.0


def test_noalloc_refuses_sizes_beyond_its_scratch():
    import torch
    we = _we()
    dev = torch.device("cuda:0")
    n_in, batch = 65, 4096               # 4096 * (65 + 258) floats > the 4096 * (64 + 258) held
    n_p = we.n_params(n_in)
    t = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device=dev)
    with pytest.raises(we.WEError) as e:
        we.mlp_loss_grad_noalloc(n_in, t(n_p), t(2 * n_in), t(batch * n_in, torch.int32), t(batch), t(1), t(n_p))
    assert e.value.status == we.WE_ECAPACITY
