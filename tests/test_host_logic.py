"""Host-side logic without a GPU: the synthetic input generators' recipes and
the denoiser workflow's bookkeeping (summary statistics, time-to-gamma
accounting, error metric)."""
import numpy as np

from paper_1409_8336_amd import denoise, synth


def test_denoiser_cases_follow_the_recipe():
    for i in (0, 7, 399):
        a = synth.denoiser_case(i)
        b = synth.denoiser_case(i)
        assert a["hu"].shape == (160, 128, 128) and a["hu"].dtype == np.int16
        np.testing.assert_array_equal(a["hu"], b["hu"])           # seeded
        np.testing.assert_array_equal(a["spots"], b["spots"])
        sp = a["spots"]
        assert sp.shape[1] == 6 and 10 <= len(sp) <= 180            # 1-3 layers x 10-60
        assert np.all((sp[:, 2] >= 70.0) & (sp[:, 2] <= 230.0))
        layers = np.unique(sp[:, 2])
        assert 1 <= len(layers) <= 3
        assert np.all(sp[:, 5] > 0)
        # titanium rod present (HU 3000), lung/soft/bone values only otherwise
        assert set(np.unique(a["hu"])) <= {-800, 0, 40, 1000, 3000}
        assert (a["hu"] == 3000).any()
    assert not np.array_equal(synth.denoiser_case(1)["hu"], synth.denoiser_case(2)["hu"])


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1e-30, 65504.0], np.float32)
    got = synth.bf16_values(synth.bf16_bits(x))
    # 8 significant bits: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 (even: 1);
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6 (even: 1 + 2^-6)
    np.testing.assert_array_equal(got[:4], [1.0, 1.0, 1.0 + 2 ** -6, -2.5])
    assert abs(got[4] - 1e-30) <= 2 ** -8 * 1e-30
    assert got[5] == 65536.0


def test_conv_weight_generator_zero_pads():
    rng = np.random.default_rng(0)
    bits, vals = synth.conv_weights(rng, 24, 16)
    assert bits.shape == (16, (27 * 24 + 31) // 32 * 32)
    assert np.all(bits[:, 27 * 24:] == 0)
    np.testing.assert_array_equal(synth.bf16_values(bits), vals)


def test_mean_relative_error_uses_the_dose_region():
    ref = np.zeros((4, 4, 4))
    ref[1:3, 1:3, 1:3] = 10.0
    ref[0, 0, 0] = 0.5                     # below 10% of the maximum: ignored
    a = ref.copy()
    a[1, 1, 1] = 11.0                      # +10% in one of 8 region voxels
    a[0, 0, 0] = 5.0
    assert abs(denoise._mean_rel_error(a, ref) - 0.1 / 8) < 1e-15


def _rec(t_low, t_inf, rates, ok, t_plain):
    return {"t_mc_low_s": t_low, "t_infer_s": t_inf, "disagreement": 0.0, "rule_fallback": False,
            "mre_denoised": 0.03, "mre_low": 0.06, "plain_wall_s": [0.001, 0.002], "plain_n": [1, 2],
            **{name: {"n_eval": 10, "gamma_pass_denoised": 0.99 if ok else 0.9,
                      "gamma_pass_low": 0.95, "plain_gamma_pass": rates, "t_plain_s": t_plain,
                      "n_plain": 2 if t_plain else None, "t_den_s": 0.0, "denoised_ok": ok,
                      "speedup": (t_plain / (t_low + t_inf + (0 if ok else t_plain))) if t_plain else None}
               for name in denoise.CRITERIA}}


def test_summary_medians_and_fallback_accounting():
    recs = [_rec(0.002, 0.001, [0.9, 0.99], True, 0.006),
            _rec(0.002, 0.001, [0.9, 0.99], False, 0.006),
            _rec(0.002, 0.001, [0.9, 0.99], True, 0.009)]
    s = denoise.summarize(recs)
    c = s["2%/2mm"]
    assert c["denoised_pass_98"] == 2 and c["cases_with_plain_reaching_98"] == 3
    # speed-ups: 0.006/0.003 = 2, 0.006/0.009 = 0.667, 0.009/0.003 = 3 -> median 2
    assert abs(c["median_speedup"] - 2.0) < 1e-12
    assert c["rule_agrees_with_gamma"] == 2      # the rule never fired; one case failed gamma
    assert abs(s["median_t_infer_ms"] - 1.0) < 1e-12
