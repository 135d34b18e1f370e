"""Host-side logic that needs no GPU: the surrogate's bookkeeping and the benchmark's byte
accounting and profile gating."""
import json
import os

import numpy as np
import pytest

import bench
from paper_2207_09334_amd import surrogate as SG


def test_standardiser_round_trip_and_constant_columns():
    rng = np.random.default_rng(0)
    a = rng.normal(3.0, 2.0, size=(500, 4))
    a[:, 2] = 7.0                                    # a constant column keeps unit scale
    s = SG.Standardiser.fit(a)
    z = s.apply(a)
    np.testing.assert_allclose(z[:, [0, 1, 3]].mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(z[:, [0, 1, 3]].std(axis=0), 1.0, rtol=1e-12)
    assert np.all(z[:, 2] == 0.0) and s.std[2] == 1.0
    np.testing.assert_allclose(s.invert(z), a, rtol=1e-12)


def test_rms_relative_error_by_hand():
    true = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 0.0]])      # RMS norm sqrt(25 / 2)
    pred = np.array([[3.0, 4.0, 1.0], [0.0, 0.0, 1.0]])      # errors of norm 1 and 1
    assert SG.rms_relative_error(pred, true) == pytest.approx(1.0 / np.sqrt(12.5))
    assert SG.rms_relative_error(true, true) == 0.0


def test_screen_takes_top_k_and_every_flagged_candidate():
    pred = np.array([[0.1, 0, 0], [0.5, 0, 0], [0.3, 0, 0], [0.9, 0, 0], [0.2, 0, 0]])
    flagged = np.array([False, False, False, False, True])
    assert SG.screen(pred, flagged, top_k=2).tolist() == [1, 3, 4]
    assert SG.screen(pred, np.zeros(5, bool), top_k=0).tolist() == []
    # ties keep input order (stable)
    assert SG.screen(np.zeros((3, 3)), np.zeros(3, bool), top_k=1).tolist() == [0]


def test_byte_counts_of_the_headline_step():
    # the explicit-incidence formula, 56 B per mass + 24 B per spring: the cantilever 400x40x40
    assert bench.formula_bytes(640_000, 8_020_476) == 228_331_424
    assert bench.formula_bytes(10, 100, actuated=True, batched=True) == 56 * 10 + 26 * 100 + 4 * 10
    # the step kernel's 16-bit entries: 58 B per mass (x and v read and written, lane map) and
    # 2 B per incidence, i.e. 4 B per spring
    assert bench.kernel_bytes(640_000, 8_020_476, "narrow") == 58 * 640_000 + 4 * 8_020_476
    assert bench.kernel_bytes(10, 100, "table", actuated=True) == 58 * 10 + 8 * 100
    assert bench.kernel_bytes(10, 100, "explicit", actuated=True) == 58 * 10 + 24 * 100


def test_profile_record_is_used_only_for_its_own_kernel_and_configuration(tmp_path, monkeypatch):
    launch = {"block_masses": 256, "batch": 4, "persistent_groups": 0, "step_form": "table"}
    rec = dict(launch, kernels_sha256=bench.kernel_source_hash(), workload="cantilever_400x40x40",
               hbm_bytes_per_launch=1.0e8, valu_wave_instr_per_launch=1.0e7)
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.profile_record("cantilever_400x40x40", launch)["hbm_bytes_per_launch"] == 1.0e8
    assert bench.profile_record("population_1024", launch) is None
    assert bench.profile_record("cantilever_400x40x40", dict(launch, block_masses=512)) is None
    path.write_text(json.dumps(dict(rec, kernels_sha256="0" * 64)))
    assert bench.profile_record("cantilever_400x40x40", launch) is None
    os.remove(path)
    assert bench.profile_record("cantilever_400x40x40", launch) is None


def test_bench_refuses_more_than_one_gpu(capsys):
    with pytest.raises(SystemExit) as e:
        bench.main(["--gpus", "2"])
    assert e.value.code != 0
    assert "one GPU" in capsys.readouterr().err


@pytest.mark.parametrize("f_true", [0.2503, 1.0062, 3.7])
def test_spectral_peak_recovers_a_known_frequency(f_true):
    """The frequency tool's FFT peak: a decaying-free sinusoid over ~6 periods with an offset,
    a weaker second harmonic and noise, sampled 200 times per period."""
    h = 1.0 / f_true / 200.0
    t = np.arange(1281) * h
    rng = np.random.default_rng(11)
    z = (0.0973 + 4e-4 * np.cos(2 * np.pi * f_true * t + 0.3) + 3e-5 * np.sin(4 * np.pi * f_true * t)
         + 2e-6 * rng.standard_normal(t.size))
    assert bench.spectral_peak(z, h) == pytest.approx(f_true, rel=2e-3)


def test_alu_roofline_cycle_count():
    """The arithmetic roofline's per-step count: 2 incidences per spring, 19 full-rate VALU
    instructions and 2 quarter-rate ones (4 cycles each) per incidence, 64 incidences per wave64
    instruction; actuated springs add 3."""
    import bench
    assert bench.alu_cycles(8_020_476) == 2 * 8_020_476 * 27 / 64
    assert bench.alu_cycles(100, actuated=True) == 2 * 100 * 30 / 64
    assert bench.VALU_PEAK == 256 * 2.4e9

