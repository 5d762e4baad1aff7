"""surr_predict_noalloc, the prediction that allocates nothing (activations in
a static device array of the library), against surr_predict on the same
network and queries, through the C ABI: two calls in a row, the second with
fewer rows, so rows the first call left in the static array must not leak
into the second."""

import numpy as np
import pytest

import parity as PT
from paper_1309_6726_amd import inputs

pytestmark = pytest.mark.gpu


def _queries(n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = inputs.surrogate_box()
    x = lo + (hi - lo) * rng.uniform(size=(n, 5))
    x[:, 2] = 10 ** rng.uniform(-4, -2, n)
    return x.astype(np.float32)


def test_predict_noalloc_matches_predict():
    import torch
    from paper_1309_6726_amd import lbm
    from paper_1309_6726_amd import surrogate as S
    net = S.Surrogate(max_batch=128, max_data=16)
    net.set_params(inputs.mlp_init_params(7))
    for n, seed in ((300, 1), (37, 2)):
        PT.say(f"[predict without allocation] {n} queries")
        x = _queries(n, seed)
        y_ref = net.predict(x)
        xd = torch.from_numpy(x).to("cuda:0")
        yd = torch.full((n, 65), float("nan"), dtype=torch.float32, device="cuda:0")
        net.predict_noalloc(xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.isfinite(y).all()
        # same kernels and per-row arithmetic: bit for bit
        assert np.array_equal(y, y_ref), float(np.abs(y - y_ref).max())
    for n in (1025, 0):
        xd = torch.zeros((max(n, 1), 5), dtype=torch.float32, device="cuda:0")
        yd = torch.zeros((max(n, 1), 65), dtype=torch.float32, device="cuda:0")
        err = lbm.lib().surr_predict_noalloc(net.h, xd.data_ptr(), n, yd.data_ptr(),
                                             net.stream.cuda_stream)
        assert err == lbm.LBM_EINVAL
    net.close()
