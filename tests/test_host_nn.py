"""Argument checks of the network-layer binding (paper_1605_00133_amd.nn) and
the learned-update set-up that run without a GPU."""

import pytest

torch = pytest.importorskip("torch")


def test_conv_rejects_bad_shapes_and_host_tensors():
    from paper_1605_00133_amd import nn
    x = torch.zeros(1, 3, 4, 4, 4)
    with pytest.raises(ValueError):
        nn.conv3d_forward(x, torch.zeros(2, 4, 3, 3, 3))        # channel mismatch
    with pytest.raises(ValueError):
        nn.conv3d_forward(x, torch.zeros(2, 3, 5, 5, 5))        # not 3x3x3
    with pytest.raises(ValueError):
        nn.conv3d_forward(x[0], torch.zeros(2, 3, 3, 3, 3))     # not 5-D
    with pytest.raises(ValueError):
        nn.conv3d_forward(x, torch.zeros(2, 3, 3, 3, 3))        # host tensors are refused
    with pytest.raises(ValueError):
        nn.conv3d_backward_input(torch.zeros(1, 5, 4, 4, 4), torch.zeros(2, 3, 3, 3, 3))
    with pytest.raises(ValueError):
        nn.relu_backward_(torch.zeros(3), torch.zeros(4))


def test_learned_update_weights_shapes():
    from paper_1605_00133_amd.learned import LearnedUpdate
    m = LearnedUpdate(n_steps=3, channels=8, seed=1, device="cpu")
    assert m.n_steps == 3
    shapes = [tuple(t.shape) for t in m.params[0]]
    assert shapes == [(8, 2, 3, 3, 3), (8,), (8, 8, 3, 3, 3), (8,), (1, 8, 3, 3, 3), (1,)]
    # the last layer starts small: the first iterates stay close to plain gradient steps
    assert float(m.params[0][4].abs().max()) < 0.3 * float(m.params[0][2].abs().max())
    m2 = LearnedUpdate(n_steps=3, channels=8, seed=1, device="cpu")
    assert all(torch.equal(a, b) for a, b in zip(m.params[2], m2.params[2]))   # seeded
