"""The ablation through libwrls on the GPU (bench.run_ablation) reproduces
the oracle's PSNR of every mode, with and without the blend, to 0.01 dB
(the outputs agree to ~1e-5 relative, which moves a PSNR by ~1e-4 dB), and
so the paper's claims hold on the GPU path too."""
import pytest

import ablation_ref
from parity import log

pytestmark = pytest.mark.gpu


def test_gpu_ablation_matches_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import bench
    W, H, T, warm = 192, 108, 30, 8
    gpu = bench.run_ablation(W, H, T, warm, sigma_s=ablation_ref.SIGMA_S,
                             sigma_r=ablation_ref.SIGMA_R, sweep=())
    ref = ablation_ref.run(W, H, T, warm)
    log("ablation gpu %s" % gpu)
    log("ablation oracle %s" % ref)
    assert abs(gpu["input"]["psnr_db"] - ref["input"]["psnr_db"]) < 0.01
    for name in ("rls_features", "wrls_features", "rls_temporal_feature", "wrls_temporal_feature",
                 "wrls_features_auto_lambda"):
        for key in ("psnr_db", "psnr_blend_db"):
            assert abs(gpu[name][key] - ref[name][key]) < 0.01, (name, key, gpu[name][key], ref[name][key])
    assert gpu["wrls_temporal_feature"]["psnr_db"] > gpu["rls_temporal_feature"]["psnr_db"]
    assert gpu["wrls_features"]["psnr_db"] > gpu["rls_features"]["psnr_db"]
