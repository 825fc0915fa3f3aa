"""GPU range-check helper: the count of pixels outside [0, T] (NaN and
infinities included) must be exact; it is integer work, compared bit for bit
with numpy."""
import numpy as np
import pytest
import torch

from paper_1105_4204_amd import synth

pytestmark = pytest.mark.gpu


def test_check_range_edge_values():
    from paper_1105_4204_amd import ops
    f = np.array([[-1.0, 0.0, 255.0, 255.5], [np.nan, np.inf, -np.inf, 128.0]], dtype=np.float32)
    assert ops.check_range(torch.from_numpy(f).cuda(), 255.0) == 5


def test_check_range_large_image_exact():
    from paper_1105_4204_amd import ops
    f = synth.piecewise_smooth(1000, 777, seed=5)
    rng = np.random.default_rng(5)
    idx = rng.choice(f.size, size=321, replace=False)
    g = f.reshape(-1).copy()
    g[idx[:100]] = -rng.uniform(1e-3, 10.0, size=100)
    g[idx[100:200]] = 255.0 + rng.uniform(1e-3, 10.0, size=100)
    g[idx[200:]] = np.nan
    g = g.reshape(f.shape)
    want = int(np.count_nonzero(~((g >= 0.0) & (g <= 255.0))))
    assert want == 321
    t = torch.from_numpy(g).cuda()
    assert ops.check_range(t, 255.0) == want
    assert ops.check_range(torch.from_numpy(f).cuda(), 255.0) == 0
    # a second call on the same stream starts from zero again
    assert ops.check_range(t, 255.0) == want
