"""Host logic of the profile summaries (paper_2308_16877_amd.profiling):
kernel-name matching, dispatch slices, the copy-probe scaling of the
traffic counters and the timed-region average of the kernel trace, on
small synthetic rocprofv3 CSV files."""
import csv
import json

from paper_2308_16877_amd import profiling as P


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_kernel_match_by_name_and_template_prefix():
    n = "void hpac::k_taf_wave<hpac::RegionBSPrice, 4, false>(hpac::KArgs, int, float, float*)"
    assert P._kernel_match(n, "k_taf_wave")
    assert not P._kernel_match(n, "k_taf")
    assert P._kernel_match("hpac::k_binomial<9, 1, true>(hpac::BoArgs)", "k_binomial<9, 1")
    assert not P._kernel_match("hpac::k_binomial<9, 2, true>(hpac::BoArgs)", "k_binomial<9, 1")


def test_dispatch_slice_keeps_dispatch_order():
    rows = [{"Dispatch_Id": str(d), "v": str(d)} for d in (7, 3, 9, 5, 11)]
    assert sorted(int(r["Dispatch_Id"]) for r in P._dispatch_slice(rows, "1:3")) == [5, 7]
    assert P._dispatch_slice(rows, None) == rows


def test_traffic_scaled_by_the_copy_probe(tmp_path):
    copy = "hpac::k_copy(float4 const*, float4*, long)"
    kern = "hpac::k_exact<hpac::RegionBSPrice, false>(hpac::KArgs)"
    kib = P.COPY_BYTES / 1024.0
    fetch = [{"Dispatch_Id": "1", "Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": str(kib / 2)},
             {"Dispatch_Id": "2", "Kernel_Name": kern, "Counter_Name": "FETCH_SIZE", "Counter_Value": "100"}]
    write = [{"Dispatch_Id": "1", "Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": str(kib)},
             {"Dispatch_Id": "2", "Kernel_Name": kern, "Counter_Name": "WRITE_SIZE", "Counter_Value": "40"}]
    _write(tmp_path / "f.csv", fetch)
    _write(tmp_path / "w.csv", write)
    out = P.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_exact", "toy",
                            str(tmp_path / "o.json"), "cf", "cw")
    # the copy reads COPY_BYTES and FETCH_SIZE saw half: scale 2; writes scale 1
    assert out["fetch"]["scale"] == 2.0 and out["write"]["scale"] == 1.0
    assert out["hbm_bytes_per_launch"] == (100 * 2 + 40) * 1024.0
    assert json.load(open(tmp_path / "o.json"))["kernel_source_sha"] == P.kernel_source_sha("k_exact")


def test_trace_summary_averages_the_timed_dispatches(tmp_path):
    name = P.STEP_KERNELS["iact"]
    stats = [{"Name": name + "(hpac::KArgs, int, float, int)", "Calls": "5", "AverageNs": "1", "MinNs": "1",
              "MaxNs": "1", "Percentage": "1"}]
    # two warm-up dispatches of 100 us, then three timed ones of 10, 20, 30 us
    trace = [{"Kernel_Name": name + "(hpac::KArgs, int, float, int)", "Start_Timestamp": "0",
              "End_Timestamp": str(int(d * 1000))} for d in (100, 100, 10, 20, 30)]
    _write(tmp_path / "s.csv", stats)
    _write(tmp_path / "t.csv", trace)
    bench = {"warmup": 1, "warmup_steps_run": 2, "steps": 3, "techniques": {"iact": {"ms": 0.025}}, "roofline": {}}
    (tmp_path / "b.json").write_text("[bench] log line\n" + json.dumps(bench) + "\n")
    P.trace_summary(str(tmp_path / "s.csv"), str(tmp_path / "t.csv"), str(tmp_path / "b.json"),
                    str(tmp_path / "o.txt"), "cmd")
    text = (tmp_path / "o.txt").read_text()
    assert "dispatches 2..4" in text
    assert "iact (%s): 20.0 (HIP events 25.0)" % name in text


def test_trace_names_with_spaced_template_closers_match():
    """A demangler that writes nested closers as "> >" names the same kernel."""
    name = "hpac::k_taf_wave<hpac::WithIo<hpac::Streamed<hpac::RegionBSPrice>>, 4, false>"
    spaced = name.replace(">>", "> >") + "(hpac::KArgs, int, float, float*)"
    assert P.short_name(spaced) == name
    assert P._kernel_match(spaced, "k_taf_wave")
