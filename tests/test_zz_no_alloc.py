"""The loss-gradient entry point that allocates nothing
(ftc_mlp_loss_grad_static), through the C ABI, against the entry point it
varies (ftc_mlp_loss_grad with a caller-owned work buffer): the same
kernels and workgroup count, so the gradient and loss must agree bit for
bit.  Two calls in a row, the second with a smaller batch (fewer partial
rows than the first call left in the shared scratch), and one with sample
indices and cube symmetries.  Seeded synthetic feature rows; the parameters
come from a seeded generator, not from training."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rows(rng, rows):
    X = np.zeros((rows, 32), np.float32)
    X[:, :27] = rng.uniform(0, 1, size=(rows, 27))
    nrm = rng.normal(size=(rows, 3))
    X[:, 27:30] = nrm / np.linalg.norm(nrm, axis=1)[:, None]
    t = (0.3 * (X[:, 14] - X[:, 12]) + 0.1 * X[:, 29]).astype(np.float32)
    return X, t


def test_static_gradient_equals_the_work_buffer_entry_point():
    import torch
    from paper_2505_06932_amd import ftc
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    rng = np.random.default_rng(77)
    theta = torch.from_numpy((0.1 * rng.normal(size=ftc.MLP_PARAMS)).astype(np.float32)).cuda()
    work = torch.zeros(ftc.MLP_WORK_FLOATS, dtype=torch.float32, device="cuda")
    # 20,000 samples fill all 256 partial rows; 700 fill 22 of them; the
    # third call picks 500 rows with symmetries
    for case, (rows, n, with_idx) in enumerate(((20000, 20000, False), (700, 700, False), (3000, 500, True))):
        _say(f"[no_alloc] call {case}: rows={rows} n={n} idx/sym={with_idx}")
        X, t = _rows(rng, rows)
        Xg, tg = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
        idx = sym = None
        if with_idx:
            idx = torch.from_numpy(rng.permutation(rows)[:n].astype(np.int32)).cuda()
            sym = torch.from_numpy(rng.integers(0, 48, size=n).astype(np.int32)).cuda()
        g_ref = torch.full((ftc.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        g_new = torch.full((ftc.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        l_ref = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        l_new = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        ftc.mlp_loss_grad(theta, Xg, tg, g_ref, work, loss=l_ref, n=n, idx=idx, sym=sym)
        ftc.mlp_loss_grad_static(theta, Xg, tg, g_new, loss=l_new, n=n, idx=idx, sym=sym)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.all(np.isfinite(a)) and np.isfinite(l_ref.item())
        assert np.array_equal(a, b), (case, float(np.abs(a - b).max()))
        assert l_ref.item() == l_new.item()
        assert np.abs(a).max() > 0.0
    # argument errors are refused on the host, before anything is launched
    with pytest.raises(ftc.FTCError):
        ftc.mlp_loss_grad_static(theta, Xg, tg, g_new, n=0)
