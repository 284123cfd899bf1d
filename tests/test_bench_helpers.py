"""Host logic of bench.py: the committed counter summaries it reads are gated
by the kernel source hash and keyed by kernel labels (which contain '=')."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _write(path, text):
    with open(path, "w") as f:
        f.write(text)


def test_valu_summary_is_read_by_label_and_gated_by_hash(tmp_path, monkeypatch):
    f = tmp_path / "valu.txt"
    monkeypatch.setattr(bench, "VALU_FILE", str(f))
    h = bench.kernel_source_hash()
    _write(f, "# a comment = with equals\nsource_hash = %s\n"
              "valu_insts_per_launch k_axis0r<float,512,tile=8> = 1234\n"
              "valu_insts_per_launch k_row_real<float,512,pad=3,block=64,pair_groups=1> = 99\n" % h)
    got = bench.measured_valu()
    assert got == {"k_axis0r<float,512,tile=8>": 1234.0,
                   "k_row_real<float,512,pad=3,block=64,pair_groups=1>": 99.0}
    _write(f, "source_hash = 0000000000000000\nvalu_insts_per_launch k_axis0r<float,512,tile=8> = 1234\n")
    assert bench.measured_valu() == {}


def test_traffic_summary_is_gated_by_kernel_and_hash(tmp_path, monkeypatch):
    f = tmp_path / "traffic_wl.txt"
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    h = bench.kernel_source_hash()
    _write(f, "kernel = k_axis0r<float,512,tile=8>\nsource_hash = %s\nhbm_bytes_per_launch = 5.5e8\n" % h)
    assert bench.measured_traffic("k_axis0r<float,512,tile=8>", "wl") == 5.5e8
    assert bench.measured_traffic("k_axis0r<float,512,tile=16>", "wl") is None
    assert bench.measured_traffic("k_axis0r<float,512,tile=8>", "other") is None
    _write(f, "kernel = k_axis0r<float,512,tile=8>\nsource_hash = x\nhbm_bytes_per_launch = 5.5e8\n")
    assert bench.measured_traffic("k_axis0r<float,512,tile=8>", "wl") is None


def test_pass_model_bytes_match_the_workload_table():
    """The pass model's bytes per step of each workload: Model A 64^2 FP64 SETD1
    0.12 MB (29.4 B per site-update), Model B 512^2 x 64 298.7 MB (17.8 B), the
    plain FP64 Model B 35.6 B, KPZ 1024^2 x 16 388.6 MB (23.2 B), CGL 256^3 x 4
    3.03 GB (45.2 B)."""
    from paper_2511_22510_amd import workloads as W
    cases = [(W.problem(W.CONFIG_A), 0.12e6, 29.4), (W.problem(W.CONFIG_B), 298.7e6, 17.8),
             (W.problem(W.CONFIG_B, precision=64, realizations=1), 9.3e6, 35.6),
             (W.problem(W.CONFIG_KPZ), 388.6e6, 23.2), (W.problem(W.CONFIG_CGL), 3.03e9, 45.2)]
    for p, step_bytes, per_site in cases:
        b = bench.survey_pass_bytes(p)
        assert len(b) == (4 if p["ndim"] == 3 else 2)
        tot = sum(b)
        sites = W.site_updates(p, 1)
        assert abs(tot / step_bytes - 1) < 0.01, (p["nl"], tot)
        assert abs(tot / sites - per_site) < 0.05, (p["nl"], tot / sites)
    # the dominant (axis-0) pass of Model B: 209.07 MB
    assert abs(bench.survey_pass_bytes(W.problem(W.CONFIG_B))[1] - 209.07e6) < 0.01e6


def test_valu_roofline_uses_the_issue_peak():
    names = ["a", "b"]
    r = bench.valu_roofline(names, [1e-5, 2e-5], 1)
    assert r["bound"] == "alu" and r["peak"] == 256 * 2.4e9
    assert r["kernel"] == "b"


def test_valu_roofline_falls_back_to_a_counted_variant(tmp_path, monkeypatch):
    f = tmp_path / "valu.txt"
    monkeypatch.setattr(bench, "VALU_FILE", str(f))
    _write(f, "source_hash = %s\n"
              "valu_insts_per_launch k_axis0r<float,512,tile=8> = 2000\n"
              "valu_insts_per_launch k_row_real<float,512,pad=3,block=256,pair_groups=1> = 1000\n"
              % bench.kernel_source_hash())
    names = ["k_row_real<float,512,pad=3,block=64,pair_groups=2>", "k_axis0r<float,512,tile=8>"]
    r = bench.valu_roofline(names, [1e-5, 2e-5], 1)
    row, ax = r["passes"]
    assert row["valu_insts_per_launch"] == 1000
    assert row["counted_variant"] == "k_row_real<float,512,pad=3,block=256,pair_groups=1>"
    assert ax["counted_variant"] == names[1] and r["achieved"] == 2000 / 2e-5


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_shipped_variant_table_parses_and_covers_the_timed_workloads(monkeypatch):
    """Every entry of the shipped table is a launch-class key and four
    variant numbers in the ranges the library accepts; the workloads the
    bench times have an entry; the bench hands the library a private copy."""
    keys = {}
    with open(bench.TUNED_TABLE) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            key, row, ax0, ax1, streams = line.split()
            assert len(key.split("|")) == 12
            assert 0 <= int(row) < 16 and 0 <= int(ax0) < 16 and 0 <= int(ax1) < 4 and int(streams) in (1, 2)
            keys[key] = int(ax0)
    # Model B 512^2 x 64 and x 256, KPZ 1024^2 x 16, CGL 256^3 x 4 (SETD2, 2/3 rule, carry storage)
    for k in ("2|0|32|1|512|512|1|0|1|0|64|1", "2|0|32|1|512|512|1|0|1|0|256|1",
              "2|0|32|1|1024|1024|1|2|1|0|16|2", "3|1|32|1|256|256|256|0|1|0|4|3"):
        assert k in keys and keys[k] >= 4   # carry storage steps with the register kernel
    monkeypatch.delenv("SETD_TUNE_CACHE", raising=False)
    path = bench.use_tuned_table()
    try:
        assert os.environ["SETD_TUNE_CACHE"] == path and path != bench.TUNED_TABLE
        assert open(path).read() == open(bench.TUNED_TABLE).read()
    finally:
        os.remove(path)
        monkeypatch.delenv("SETD_TUNE_CACHE", raising=False)


def test_event_gap_is_subtracted_only_for_one_stream():
    """The dispatch gap the per-pass events add is the bracketed sum less the
    uninstrumented step time on one stream; a plan stepping on two streams
    overlaps its halves in the uninstrumented step, so its brackets stand."""
    import numpy as np
    from paper_2511_22510_amd import workloads as W
    p = W.problem(W.CONFIG_B)

    class Info:
        pass

    def run(streams):
        info = Info()
        info.streams = streams
        info.pass_bytes = [1e8, 2e8, 0.0, 0.0]
        prof = np.array([[2.5, 100.0], [4.0, 100.0]])   # 25 and 40 us per launch
        r = dict(info=info, ev=100 * 60e-6, steps=100, prof=prof)   # 60 us per plain step
        return bench.pass_roofline(r, p, ["row", "axis0"])[0]

    one, two = run(1), run(2)
    assert one["kernel"] == two["kernel"] == "axis0"
    assert abs(one["event_gap_us"] - 2.5) < 1e-9 and abs(one["avg_launch_us"] - 37.5) < 1e-9
    assert two["event_gap_us"] == 0.0 and abs(two["avg_launch_us"] - 40.0) < 1e-9
    assert one["step_streams"] == 1 and two["step_streams"] == 2
