"""Host-side logic of bench.py (no GPU): the one-GPU contract and the
algorithmic byte model the roofline divides by."""
import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2", "--steps", "1"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def test_traffic_model_matches_the_documented_figures():
    # the per-launch algorithmic bytes quoted for 127^3 FP64 (6 levels,
    # constant coefficients) in the design notes' kernel table
    m, per_iter = bench.traffic_model(3, 127, 6, 8, False)
    assert round(m["update_xP"] / 1e6, 1) == 255.8
    assert round(m["spmm_gram"] / 1e6, 1) == 213.0
    assert round(m["update_r"] / 1e6, 1) == 131.1
    assert round(m["fine_W"] / 1e6, 1) == 124.7
    # FP32 bulk halves the block traffic; x and r stay FP64
    m32, per32 = bench.traffic_model(3, 127, 6, 4, False)
    assert m32["update_r"] == (6 * 4 + 16) * 127 ** 3 and per32 < per_iter


def test_poisson_csr_inputs_match_the_structured_hierarchy():
    """The CSR inputs bench.py builds for the general entry point are the
    structured workload's operator and prolongations (compared with the
    oracle's own construction at 15^3, 3 levels)."""
    from oracle import hierarchy
    A, Ps = bench.poisson_csr(15, 3)
    h = hierarchy.build(3, 15, 3)
    assert abs(A - h.fine.A).max() <= 1e-12 * abs(h.fine.A).max()
    for l in range(2):
        assert Ps[l].shape == h.levels[l].P.shape
        assert abs(Ps[l] - h.levels[l].P).max() == 0.0


def test_x1_fields_and_host_description():
    """The mixed-precision error fields and the CPU description of the
    baseline (host only)."""
    import numpy as np
    x64 = np.linspace(1.0, 2.0, 100)
    x32 = x64 * (1.0 + 1e-7)
    f = bench.x1_fields(x32, {"relres_true": 5e-9}, x64, 16)
    assert abs(f["err_vs_fp64"] - 1e-7) <= 1e-9
    assert f["iterations_fp64"] == 16 and f["relres_true"] == 5e-9
    assert bench.rel_err(x64, x64) == 0.0
    assert bench.host_threads() >= 1
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_unet_work_counts():
    """The U-Net's work at 128^3 on the padded channel counts and on the real
    ones (w1: 2 of 16 input channels, w11: 1 of 16 outputs)."""
    import bench
    gp, gu = bench.unet_gflop(128), bench.unet_gflop(128, padded=False)
    assert abs(gp - 265.6) < 0.05 and abs(gu - 239.2) < 0.05
    line = bench.unet_line(0.5, 128)
    assert line["gflop"] == round(gu, 1) and abs(line["bf16_peak_frac"] - gu / 0.5 / 2500.0) < 1e-4
