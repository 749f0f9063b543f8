"""Host-side pieces of the measurement path (no GPU): the source digests that
tie a committed HBM-traffic report to the kernel it was taken on, and the
report reader the bench uses."""
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
