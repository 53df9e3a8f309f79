"""Host logic of the rocprofv3 summariser: kernel-name shortening, counter
calibration against the copy dispatch, and the source fingerprint check."""
import os

from paper_1111_0716_amd import profile_summary as ps

HDR = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
       '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
       '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "p_counter_collection.csv"), "w") as f:
        f.write(HDR)
        for i, (name, val) in enumerate(rows):
            f.write(f'{i},{i},"Agent 1",1,1,1,64,1,"{name}",64,0,0,8,0,8,"{counter}",{val},0,1\n')


def test_short_name():
    assert ps.short_name("void fock::k_pair_fused<float, 32>(int, long long)") == "fock::k_pair_fused<float, 32>"
    assert ps.short_name("void fock::(anonymous namespace)::k_overlap_mfma<double>(double const*)") == \
        "fock::k_overlap_mfma<double>"
    assert ps.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_traffic_calibration_and_fingerprint(tmp_path):
    kern = "void fock::k_pair_fused<float, 32>(int)"
    # the copy of 1 MiB reads as 512 KiB (factor 2) and writes as 1024 KiB (factor 1)
    _write(str(tmp_path / "f"), "FETCH_SIZE", [(ps.COPY_KERNEL, 512.0), (ps.COPY_KERNEL, 1.0), (kern, 999.0),
                                               (kern, 100.0), (kern, 300.0)])
    _write(str(tmp_path / "w"), "WRITE_SIZE", [(ps.COPY_KERNEL, 1024.0), (kern, 5.0), (kern, 50.0)])
    out = tmp_path / "t.md"
    ps.main(["traffic", "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--kernel",
             "k_pair_fused<float, 32>", "--kind", "fused", "--copy-bytes", str(1 << 20), "--units-per-launch", "2",
             "--bytes-per-unit", "1024", "--title", "t", "--command", "c", "--out", str(out)])
    # first dispatch dropped: fetch mean 200 KiB x 2, write 50 KiB x 1
    want = (200 * 2 + 50) * 1024.0
    got = ps.read_traffic(str(out), "fused")
    assert abs(got - want) <= 1e-6 * want
    assert ps.read_traffic(str(out), "plane") is None
    text = out.read_text().replace(ps.sources_sha256("fused"), "0" * 64)
    out.write_text(text)
    assert ps.read_traffic(str(out), "fused") is None
    assert ps.read_traffic(str(tmp_path / "absent.md"), "fused") is None


def test_counter_summary_means_and_derived_shares(tmp_path):
    kern = "void fock::k_pair_fused<float, 32>(int)"
    _write(str(tmp_path / "a"), "SQ_WAVE_CYCLES", [(kern, 10.0), (kern, 1000.0), (kern, 3000.0)])
    d = str(tmp_path / "a" / "p_counter_collection.csv")
    with open(d, "a") as f:
        for i, v in enumerate((5.0, 500.0, 1500.0)):
            f.write(f'{10 + i},{10 + i},"Agent 1",1,1,1,64,1,"{kern}",64,0,0,8,0,8,"SQ_ACTIVE_INST_VALU",{v},0,1\n')
    text = ps.counters_summary([str(tmp_path / "a")], "k_pair_fused<float, 32>", "t", ["c"])
    assert "| SQ_WAVE_CYCLES | 2.0000e+03 |" in text
    assert "VALU issuing: 50.0 % of wave cycles" in text
