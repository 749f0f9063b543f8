"""Host-side pieces of the measurement path (no GPU): the source digests that
tie a committed HBM-traffic report to the kernel it was taken on, the report
reader the bench uses, the summary modes on synthetic counter CSV, and the
bench's refusal of more than one GPU."""
import os

from paper_1703_05638_amd import profile_summary as ps


def test_every_digest_region_is_found_in_the_kernel_source():
    # the bench reads a traffic report only through these digests: a region
    # marker that went missing from kernels.hip would break every bench run
    for key in ps.KERNEL_SOURCES:
        d = ps.source_digest(key)
        assert len(d) == 16 and int(d, 16) >= 0


def test_report_is_read_only_while_its_kernel_source_is_unchanged(tmp_path):
    digest = ps.source_digest("k_gram")
    good = tmp_path / "good.txt"
    good.write_text("# header\nkernel_regex: k_gram_mfma\nkernel_source_sha256_16: %s\n"
                    "traffic_bytes_per_launch: 1234.5\n" % digest)
    assert ps.read_traffic(str(good)) == 1234.5
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_regex: k_gram_mfma\nkernel_source_sha256_16: 0000000000000000\n"
                     "traffic_bytes_per_launch: 1234.5\n")
    assert ps.read_traffic(str(stale)) is None
    assert ps.read_traffic(str(tmp_path / "absent.txt")) is None


def test_digest_keys_follow_the_kernel_regex():
    assert ps._source_key("k_gram_mfma") == "k_gram"
    assert ps._source_key("k_proj_mfma") == "k_proj"
    assert ps._source_key("k_mg_up<float") == "k_mg"
    assert ps._source_key("k_cheb<float") == "k_cheb"
    assert ps._source_key("k_sine_x1") == ps._source_key("k_tridiag_x2") == "k_cd"
    # the multigrid kernels share one region, so both reports follow it
    assert ps.source_digest("k_mg") == ps.source_digest(ps._source_key("k_mg_down<float"))


def test_committed_reports_name_their_kernels():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prof = os.path.join(root, "profiles")
    for name in os.listdir(prof):
        if not name.endswith("_traffic.txt"):
            continue
        text = open(os.path.join(prof, name)).read()
        assert "kernel_regex:" in text and "traffic_bytes_per_launch:" in text
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text


def test_bench_kernel_table_matches_the_library_kinds():
    import bench
    from paper_1703_05638_amd import lrpost as lp

    kinds = {lp.LRPOST_KERNEL_SMOOTHER_STEP: "k_cheb", lp.LRPOST_KERNEL_MG_DOWN: "k_mg_down",
             lp.LRPOST_KERNEL_MG_UP: "k_mg_up", lp.LRPOST_KERNEL_GRAM: "k_gram_mfma",
             lp.LRPOST_KERNEL_PROJ: "k_proj_mfma", lp.LRPOST_KERNEL_STENCIL: "k_stencil_strip",
             lp.LRPOST_KERNEL_GRAM32: "k_gram_f32", lp.LRPOST_KERNEL_PROJ32: "k_proj_grouped_f32"}
    assert {k: v[0] for k, v in bench.KERNELS.items()} == kinds
    # the dominant kernel's committed traffic reports exist under the names the bench looks for
    for name in ("k_gram_mfma", "k_mg_up", "k_mg_down"):
        assert os.path.exists(bench.traffic_report(name, "mixed", "mesh1024_nt1000"))


def _write_counters(d, rows):
    import csv
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_counter_sums_per_kernel_regex(tmp_path, capsys):
    """The counters mode sums each counter over the dispatches a regex
    matches (several rows of one dispatch, e.g. one per XCD, add up); the
    regexes are separated by ';' so that a template argument list with a
    comma stays one regex."""
    _write_counters(tmp_path, [
        (1, "void k_gram_mfma<3, 2>(long)", "SQ_WAVES", 2), (1, "void k_gram_mfma<3, 2>(long)", "SQ_WAVES", 3),
        (2, "void k_gram_mfma<1, 1>(long)", "SQ_WAVES", 7), (3, "k_proj_grouped(x)", "SQ_WAVES", 11),
        (1, "void k_gram_mfma<3, 2>(long)", "SQ_BUSY_CYCLES", 100),
    ])
    ps.counters(str(tmp_path), "k_gram_mfma<3, 2>;k_gram_mfma;k_proj_grouped\\(")
    out = capsys.readouterr().out.splitlines()
    assert out[0] == "k_gram_mfma<3, 2>: dispatches 1"
    assert "SQ_BUSY_CYCLES sum 1.000000e+02" in out[1] and "SQ_WAVES sum 5.000000e+00" in out[2]
    assert out[3] == "k_gram_mfma: dispatches 2"
    assert "SQ_WAVES sum 1.200000e+01" in out[5]
    assert out[6] == "k_proj_grouped\\(: dispatches 1"
    assert "SQ_WAVES sum 1.100000e+01" in out[8]


def test_traffic_scales_each_counter_by_the_copy(tmp_path, capsys):
    """traffic divides the kernel's mean FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) by what each counter reads for the copy of known size."""
    f, w = tmp_path / "f", tmp_path / "w"
    f.mkdir()
    w.mkdir()
    copy = 1 << 20  # bytes each way
    # the copy: FETCH reads half its bytes, WRITE all of them
    _write_counters(f, [(1, "MulFunctor", "FETCH_SIZE", copy / 2048), (2, "k_x", "FETCH_SIZE", 100.0),
                        (3, "k_x", "FETCH_SIZE", 300.0)])
    _write_counters(w, [(1, "MulFunctor", "WRITE_SIZE", copy / 1024), (2, "k_x", "WRITE_SIZE", 10.0),
                        (3, "k_x", "WRITE_SIZE", 30.0)])
    ps.traffic(str(f), str(w), "k_x", "MulFunctor", copy)
    vals = dict(line.split(": ", 1) for line in capsys.readouterr().out.splitlines())
    assert float(vals["fetch_scale_factor"]) == 0.5 and float(vals["write_scale_factor"]) == 1.0
    # (200 KiB / 0.5 + 20 KiB / 1.0) per launch
    assert float(vals["traffic_bytes_per_launch"]) == (400.0 + 20.0) * 1024


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU: --gpus 2 ends with status 2 and says so,
    before any device work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
