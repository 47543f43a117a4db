"""snk_mlp_loss_grad_noalloc (the entry point for callers that cannot allocate device memory)
against snk_mlp_loss_grad through the C ABI: same kernels, so the gradients and the loss
agree bitwise, on two calls in a row, the second with fewer samples (the fixed scratch array
keeps the first call's partial sums, which the second must not pick up); more samples than
the array holds is an argument error.  The gradient itself is checked against the FP64
reference in test_gpu_mlp.py."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _net(seed):
    import torch
    from paper_2303_14280_amd import snk
    from oracle import mlp_ref
    rng = np.random.default_rng(seed)
    m = snk.Mlp(0)
    m.set_params(mlp_ref.flatten(mlp_ref.init_params(seed)).astype(np.float32))
    m.set_normalisation(rng.normal(size=16).astype(np.float32), rng.uniform(0.5, 2.0, size=16).astype(np.float32))
    return m


def _data(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.normal(size=(n, 16)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    return X, t


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    import torch
    from paper_2303_14280_amd import snk
    m = _net(7)
    for call, n in enumerate((50000, 3000)):
        X, t = _data(n, 100 + call)
        g_ref = torch.full((m.nparams + 1,), float("nan"), dtype=torch.float32, device="cuda")
        g_new = torch.full((m.nparams + 1,), float("nan"), dtype=torch.float32, device="cuda")
        print("no-alloc call", call, "samples", n, flush=True)
        m.loss_grad(X.data_ptr(), t.data_ptr(), n, g_ref.data_ptr(), under=10.0)
        m.loss_grad_noalloc(X.data_ptr(), t.data_ptr(), n, g_new.data_ptr(), under=10.0)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))


def test_noalloc_rejects_more_samples_than_the_scratch_array():
    import torch
    from paper_2303_14280_amd import snk
    m = _net(8)
    n = 65536 + 64
    X, t = _data(n, 3)
    g = torch.zeros(m.nparams + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(snk.SnkError) as ei:
        m.loss_grad_noalloc(X.data_ptr(), t.data_ptr(), n, g.data_ptr())
    assert ei.value.status == snk.SNK_E_ARG and "65536" in str(ei.value)
    # the largest accepted size runs
    m.loss_grad_noalloc(X.data_ptr(), t.data_ptr(), 65536, g.data_ptr())
    torch.cuda.synchronize()
    assert np.all(np.isfinite(g.cpu().numpy()))
