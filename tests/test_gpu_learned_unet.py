"""The learned reconstruction at the paper-scale workload against plain TV-Bregman.

128^3, Nt = 740, 12.5 % scrambled-Hadamard sub-sampling (2048 of 16384 patterns),
24-vessel phantoms with 1 % noise; the committed U-Net weights
(paper_1605_00133_amd/weights/, trained by `python -m paper_1605_00133_amd.learned_unet`
on TV+Br reconstructions of phantoms 1000-1071) on held-out phantoms 5004-5007
(never used in training or in choosing the model). For each, plain TV+Br
(5 x 50 FISTA, lambda_Br = 10 lambda_TV+ from the discrepancy principle) logs PSNR
and time per iteration; its target is its final PSNR minus 0.5 dB. The learned
iteration (8 unrolled steps, with its fallback check against plain FISTA at equal
pairs running concurrently) is asserted to
* need no fallback (its data residual below plain FISTA's at the same pairs);
* take at least 5x less wall time than TV+Br needs to reach its target;
* end within 0.5 dB of the final TV+Br PSNR on average (on the validation phantoms
  5000-5003, used to pick the model: 0.38 dB below on average, 0.24-0.54 dB per
  phantom);
* be more than 1 dB above the PSNR TV+Br has reached after the same wall time: the
  gain of the trained network over the method without it.
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_STEPS = 8


def test_learned_unet_against_tvbr_time_to_target():
    from paper_1605_00133_amd import pat as P
    from paper_1605_00133_amd.learned_unet import (LearnedUNetRecon, evaluate_case, make_case, make_plan,
                                                   summarize, weights_path)
    from gpu_cases import to_dev
    from synthetic import gaussian_volume
    path = weights_path(128, "hadamard")
    assert os.path.exists(path), f"committed weights {path} are missing"
    model = LearnedUNetRecon.load(path).truncated(N_STEPS)
    plan = make_plan(128, "hadamard")
    ref_plan = make_plan(128, "hadamard")
    L = P.pat_power_iteration(plan, to_dev(gaussian_volume(plan.vol_shape, 8)), 10)
    rows = []
    for seed in (5004, 5005, 5006, 5007):
        case = make_case(plan, seed, "hadamard")
        rows.append(evaluate_case(model, plan, case, L, ref_plan=ref_plan))
        r = rows[-1]
        print(f"phantom {seed}: TV+Br {r['tvbr_final_db']:.2f} dB (target {r['tvbr_target_db']:.2f} dB at "
              f"{r['tvbr_t_target_ms']:.0f} ms, all 250 iterations {r['tvbr_total_ms']:.0f} ms); learned "
              f"{r['learned_db']:.2f} dB in {r['learned_ms']:.0f} ms: {r['db_vs_tvbr']:+.2f} dB, "
              f"{r['speedup_vs_target_time']:.1f}x; TV+Br after the same time {r['tvbr_db_at_learned_time']:.2f} dB; "
              f"fallback {r['fallback']}")
    s = summarize(rows)
    print({k: v for k, v in s.items()})
    assert s["fallbacks"] == 0
    assert s["mean_speedup_vs_target_time"] >= 5.0
    assert s["mean_db_vs_tvbr"] >= -0.5
    assert all(r["gain_vs_tvbr_same_time"] > 1.0 for r in rows)
    assert np.isfinite(s["mean_learned_db"])
    ref_plan.close()
    plan.close()
