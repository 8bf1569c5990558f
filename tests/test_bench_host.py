"""Host logic of bench.py: the measured-traffic figures it reports are built
only from rocprofv3 summaries taken on the current kernel sources."""
import os
import shutil

import bench


def test_step_hbm_sums_the_kernels_of_the_timed_steps(monkeypatch):
    vals = {"pc": 200e9, "zinv": 65e9, "theta": 58e9, "zfwd": 32e9, "curl": 26e9}
    monkeypatch.setattr(bench, "read_traffic", lambda k, w, p: vals[k])
    # 10 timed steps; the curl was not launched in them (formed by the last sweep)
    times = {"pc": (36.0, 10), "curl": (0.0, 0), "zinv": (12.0, 10), "theta": (20.0, 10), "zfwd": (6.0, 10)}
    r = bench.step_hbm(times, 10, 0.75, "production", "fp64")
    assert r["bytes_per_step"] == int(355e9)
    assert abs(r["achieved_GBs"] - 355e9 / 0.075 / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved_GBs"] / bench.HBM_PEAK_GBS) < 1e-4
    assert "curl" not in r["bytes_per_step_by_kernel"]
    # a kernel launched twice per step counts twice
    times["zinv"] = (6.0, 20)
    r2 = bench.step_hbm(times, 10, 0.75, "production", "fp64")
    assert r2["bytes_per_step"] == int(355e9 + 65e9)


def test_step_hbm_is_none_without_every_summary(monkeypatch):
    vals = {"pc": 200e9, "zinv": 65e9, "theta": None, "zfwd": 32e9, "curl": 26e9}
    monkeypatch.setattr(bench, "read_traffic", lambda k, w, p: vals[k])
    times = {"pc": (36.0, 1), "curl": (0.0, 0), "zinv": (12.0, 1), "theta": (20.0, 1), "zfwd": (6.0, 1)}
    assert bench.step_hbm(times, 1, 0.075, "production", "fp64") is None


def test_read_traffic_checks_the_source_digest(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_1311_2481_amd", "csrc")
    dst = tmp_path / "paper_1311_2481_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES["zinv"]:
        shutil.copy(os.path.join(src, name), dst / name)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.source_digest("zinv")
    (tmp_path / "profiles" / "traffic_zinv_w_fp64.txt").write_text(
        f"# header\nsource_sha = {sha}\nbytes_per_launch = 123456\n")
    assert bench.read_traffic("zinv", "w", "fp64") == 123456.0
    assert bench.read_traffic("zinv", "w", "fp32_bulk") is None  # no summary
    # any change to a source the kernel is built from voids the summary
    with open(dst / bench.KERNEL_SOURCES["zinv"][0], "a") as fh:
        fh.write("\n")
    assert bench.read_traffic("zinv", "w", "fp64") is None


def test_algorithmic_bytes_of_the_production_step():
    """B_alg = 256 B of state per stored slot-row (read u^i, u^{i-1}, N^i,
    N^{i-1}; write u^{i+1}, p) plus the factors of the 4 operators, 9
    doubles per row of every distinct mode, read once: 400 S bytes with
    S = N_r m_theta m_z (107.4 GB at N_r = 512, 512 x 1024 modes)."""
    import tc_inputs
    cfg = tc_inputs.Config(tc_inputs.CONFIGS["production"])
    S = cfg.n_r * cfg.m_theta * cfg.m_z
    assert bench.step_alg_bytes(cfg) == 400 * S == 107374182400
    kb = bench.kernel_bytes(cfg, "fp64")
    assert kb["pc"] == bench.step_alg_bytes(cfg)
    spec = cfg.m_theta * (cfg.m_z - 1) * 16
    inter = (3 * cfg.m_z // 2) * cfg.m_theta * 16
    assert kb["zinv"] == (6 * spec + 6 * inter) * cfg.n_r
    assert kb["theta"] == 9 * inter * cfg.n_r
    assert kb["zfwd"] == (3 * inter + 3 * spec) * cfg.n_r
    # FP32-bulk halves the intermediate only
    k32 = bench.kernel_bytes(cfg, "fp32_bulk")
    assert k32["theta"] * 2 == kb["theta"] and k32["pc"] == kb["pc"]
