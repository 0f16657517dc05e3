"""The paper's qualitative claims about its design (Sec. 5.3, Fig. 8-9),
reproduced on a seeded synthetic sequence with the FP64 oracle: the
weighted RLS beats plain RLS (supplied features, and the paper's temporal
feature with the Eq. 13 weight), the 5x5 blend of neighbour-model
predictions improves on the temporal output, and every mode improves on the
noisy input by far.  Margins are about half of the measured gaps (0.9 dB,
1.2 dB and 7 dB at 160x90 and 192x108, 30 frames)."""
import ablation_ref


def test_weighted_rls_blend_and_denoising_claims():
    res = ablation_ref.run(160, 90, 30, 8)
    inp = res["input"]["psnr_db"]
    for name in ("rls_features", "wrls_features", "rls_temporal_feature", "wrls_temporal_feature"):
        r = res[name]
        assert r["psnr_db"] > inp + 5.0, (name, r, inp)
        assert r["psnr_blend_db"] > r["psnr_db"] + 0.5, (name, r)
    assert res["wrls_features"]["psnr_db"] > res["rls_features"]["psnr_db"] + 0.4, res
    assert res["wrls_temporal_feature"]["psnr_db"] > res["rls_temporal_feature"]["psnr_db"] + 0.4, res
