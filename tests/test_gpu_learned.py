"""The learned update step (paper_1605_00133_amd.learned) on synthetic 32^3 data:
trained on plain TV+Br reconstructions, it must beat plain TV+ FISTA run for
the same number of operator pairs on held-out phantoms (PSNR, eq. PSNR). Its
distance to the TV+Br PSNR and the wall-time ratio are printed, not asserted."""

import pytest

pytestmark = pytest.mark.gpu


def test_learned_update_beats_plain_fista_with_equal_pairs():
    from paper_1605_00133_amd.learned import experiment
    out = experiment(n=32, n_train=16, n_test=4, n_steps=4, epochs=80, log=print)
    print(out)
    assert out["train_mse"][-1] < out["train_mse"][0]
    assert out["psnr_db_learned_minus_plain"] > 1.0
