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


def test_unet_recon_save_load_roundtrip(tmp_path):
    """Saved models keep their step count and widths; convolution weights are stored as
    bfloat16 (what the matrix cores multiply), biases as float32."""
    from paper_1605_00133_amd.learned_unet import LearnedUNetRecon
    m = LearnedUNetRecon(n_steps=3, widths=(4, 8, 8), seed=2, device="cpu")
    for k, net in enumerate(m.nets):
        net.params["c1"][1].fill_(0.25 + k)
    path = str(tmp_path / "m.safetensors")
    m.save(path)
    r = LearnedUNetRecon.load(path, device="cpu")
    assert r.n_steps == 3 and r.widths == (4, 8, 8) and r.n_params == m.n_params
    for a, b in zip(m.nets, r.nets):
        for name in a.params:
            assert torch.equal(b.params[name][0], a.params[name][0].to(torch.bfloat16).float())
            assert torch.equal(b.params[name][1], a.params[name][1])
    assert r.truncated(2).n_steps == 2
    with pytest.raises(ValueError):
        r.truncated(4)


def test_continued_training_checks_before_any_device_work(tmp_path):
    """Training phantoms may not reach the held-out seeds, and a starting model must have at
    least the asked-for steps of the same widths; both are refused before anything runs."""
    from paper_1605_00133_amd.learned_unet import LearnedUNetRecon, experiment, initial_model
    with pytest.raises(ValueError):
        experiment(n_train=24, train_seed0=4990)
    with pytest.raises(ValueError):
        experiment(n_train=4, train_seed0=-1)
    path = str(tmp_path / "m.safetensors")
    LearnedUNetRecon(n_steps=3, widths=(4, 8, 8), seed=0, device="cpu").save(path)
    assert initial_model(2, (4, 8, 8), path, "cpu").n_steps == 2
    with pytest.raises(ValueError):
        initial_model(4, (4, 8, 8), path, "cpu")       # more steps than saved
    with pytest.raises(ValueError):
        initial_model(2, (4, 8, 16), path, "cpu")      # other widths
    assert initial_model(2, (4, 8, 8), None, "cpu").n_steps == 2


def test_psnr_at_time_takes_last_logged_iteration():
    import numpy as np
    from paper_1605_00133_amd.learned_unet import psnr_at_time
    ref = {"_psnr": np.array([10.0, 12.0, 15.0]), "_t_ms": np.array([100.0, 200.0, 300.0])}
    assert psnr_at_time(ref, 250.0) == 12.0
    assert psnr_at_time(ref, 300.0) == 15.0
    assert psnr_at_time(ref, 99.0) == float("-inf")
