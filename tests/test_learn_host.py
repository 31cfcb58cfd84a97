"""Host-side logic of the learned-ordering pipeline (no GPU): label
centring and the zero weight of constant features."""
import numpy as np
import torch

from paper_1909_09213_amd import learn


def test_centre_labels_per_group():
    r = torch.zeros(7, 8)
    r[:, 6] = torch.tensor([0, 0, 0, 1, 1, 1, 1.])   # node / instance id
    r[:, 5] = torch.tensor([2, 2, 3, 2, 2, 2, 2.])   # depth
    r[:, 7] = torch.tensor([1, 3, 5, 2, 4, 6, 8.])
    c = learn.centre_labels(r)
    assert torch.allclose(c[:, 7], torch.tensor([-1., 1., 0., -3., -1., 1., 3.]))
    assert torch.equal(c[:, :7], r[:, :7])  # only the label column changes


def test_centring_keeps_the_order_within_a_group():
    rng = np.random.default_rng(0)
    r = torch.from_numpy(rng.uniform(0, 1, (50, 8)).astype(np.float32))
    r[:, 6] = torch.from_numpy(rng.integers(0, 5, 50).astype(np.float32))
    r[:, 5] = 1.0
    c = learn.centre_labels(r)
    for g in range(5):
        m = r[:, 6] == g
        if m.sum() > 1:
            assert torch.equal(torch.argsort(r[m, 7]), torch.argsort(c[m, 7]))
            assert abs(float(c[m, 7].sum())) < 1e-4


def test_init_theta_shape_and_scale():
    th = learn.init_theta(3)
    assert th.shape == (449,) and th.dtype == np.float32
    assert np.all(th[320:384] == np.float32(0.01)) and th[448] == 0.0
