"""rsur_forward_static (the surrogate's forward for callers that cannot allocate, members' outputs in
a fixed device array) against rsur_forward on the same context, through the C ABI: bit for bit on
two calls in a row, the second with fewer rows, plus the FP64 oracle at the BF16 bound of the
surrogate tests, and the size limit rejected with an error."""
import numpy as np
import pytest

from oracle import surrogate as S
from synth.surrogate import init_params

pytestmark = pytest.mark.gpu

DIMS = dict(din=153, width=256, depth=4, dout=6)
K = 5


def test_static_forward_equals_forward_on_two_calls():
    import torch
    from paper_1902_09171_amd import rcell, rsur
    rsur.load()
    net = rsur.Surrogate(ensemble=K, max_batch=1024, **DIMS)
    params = [init_params(net.dims, 23, k) for k in range(K)]
    for k, p in enumerate(params):
        net.set_params(k, p)
    rng = np.random.default_rng(5)
    x_mu, x_sd = rng.normal(0, 1, 153), rng.uniform(0.5, 2, 153)
    y_mu, y_sd = rng.normal(0, 1, 6), rng.uniform(0.5, 2, 6)
    net.set_norm(x_mu, x_sd, y_mu, y_sd)
    for B in (1000, 300):                        # the second call is smaller than the first
        X = rng.normal(x_mu, x_sd, (B, 153))
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda:0")
        outs = []
        for fn in (net.forward, net.forward_static):
            mean = torch.full((B, 6), float("nan"), device="cuda:0")
            var = torch.full((B, 6), float("nan"), device="cuda:0")
            fn(Xd.data_ptr(), B, mean.data_ptr(), var.data_ptr())
            torch.cuda.synchronize()
            outs.append((mean.cpu().numpy(), var.cpu().numpy()))
        (m0, v0), (m1, v1) = outs
        print(f"B={B}: max |mean diff| {np.abs(m1 - m0).max():.3e}, max |var diff| {np.abs(v1 - v0).max():.3e}",
              flush=True)
        assert np.all(np.isfinite(m1)) and np.all(np.isfinite(v1))
        assert np.array_equal(m0, m1) and np.array_equal(v0, v1)
        m_ref, v_ref = S.ensemble_predict(params, net.dims, X, x_mu, x_sd, y_mu, y_sd)
        assert np.abs(m1 - m_ref).max() <= 1e-2 * np.abs(m_ref).max()
    # beyond the fixed array: 5 members x 8192 rows x 64 padded outputs > 2^21 floats
    big = 8192
    Xb = torch.zeros((big, 153), device="cuda:0")
    mb = torch.zeros((big, 6), device="cuda:0")
    with pytest.raises(rcell.RCellError):
        net.forward_static(Xb.data_ptr(), big, mb.data_ptr())
    with pytest.raises(rcell.RCellError):
        net.forward_static(Xb.data_ptr(), 0, mb.data_ptr())
    net.close()
