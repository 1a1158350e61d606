"""The rocprofv3 summary reader that bench.py uses for its roofline figures
(paper_0912_4506_amd/profiling.py), on synthetic CSV files of the layout
rocprofv3 writes: kernel times (median), HBM bytes from FETCH_SIZE and
WRITE_SIZE scaled by the copy kernel's reading, SQ counters per launch, the
Markdown round trip, and the kernel-source hash that marks a summary stale."""
import csv
import os

import pytest

from paper_0912_4506_amd import profiling


def write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


K = "void jac::tblock_kernel<double, 4, 1, 6, 12, 0>(jac::TbArgs<double>)"
COPY = "jac::copy_kernel(HIP_vector_type<unsigned int, 4u> const*, HIP_vector_type<unsigned int, 4u>*, long)"


@pytest.fixture()
def runs(tmp_path):
    trace = [{"Kernel_Name": K, "Start_Timestamp": 1000 * i, "End_Timestamp": 1000 * i + d}
             for i, d in enumerate([520000, 530000, 900000, 525000, 528000])]
    trace += [{"Kernel_Name": COPY, "Start_Timestamp": 0, "End_Timestamp": 700000}]
    write_csv(str(tmp_path / "trace/host/123_kernel_trace.csv"), trace)
    for name, counter, kval, cval in (("fetch", "FETCH_SIZE", 600000.0, 1048576.0),
                                      ("write", "WRITE_SIZE", 1050000.0, 2097152.0)):
        rows = [{"Dispatch_Id": d, "Kernel_Name": K, "Counter_Name": counter, "Counter_Value": kval / 2}
                for d in (1, 1)]          # two rows of one dispatch are summed
        rows += [{"Dispatch_Id": 2, "Kernel_Name": COPY, "Counter_Name": counter, "Counter_Value": cval}]
        write_csv(str(tmp_path / f"{name}/host/9_counter_collection.csv"), rows)
    sq = [{"Dispatch_Id": 1, "Kernel_Name": K, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 1.5e8},
          {"Dispatch_Id": 1, "Kernel_Name": K, "Counter_Name": "SQ_INSTS_LDS", "Counter_Value": 7e6}]
    write_csv(str(tmp_path / "sq/host/9_counter_collection.csv"), sq)
    return tmp_path


def test_summary_figures(runs):
    d = str(runs)
    fig = profiling.summarize("tblock_kernel<double, 4, 1, 6, 12, 0>", d + "/trace", d + "/fetch",
                              d + "/write", d + "/sq")
    assert fig["launches"] == 5 and fig["median_us"] == 528.0
    # FETCH: 2 GiB copy reads as 1048576 KiB -> scale 2; WRITE reads 2097152 -> scale 1
    assert fig["fetch_scale"] == 2.0 and fig["write_scale"] == 1.0
    assert fig["fetch_gb_per_launch"] == round(600000 * 1024 * 2 / 1e9, 4)
    assert fig["traffic_gb_per_launch"] == round(fig["fetch_gb_per_launch"] + fig["write_gb_per_launch"], 4)
    assert fig["sq_insts_valu_per_launch"] == 150000000
    path = str(runs / "summary.md")
    profiling.write_summary(path, dict(fig), "title", ["rocprofv3 ..."])
    back = profiling.read_figures(path)
    assert back["traffic_gb_per_launch"] == fig["traffic_gb_per_launch"]
    assert back["kernel"] == K and back["kernel_source_sha"] == profiling.kernel_source_hash()
    assert profiling.read_figures(str(runs / "missing.md")) == {}


def test_ambiguous_kernel_is_an_error(runs):
    with pytest.raises(KeyError):
        profiling.summarize("kernel", trace=str(runs / "trace"))


def test_source_hash_is_stable():
    assert profiling.kernel_source_hash() == profiling.kernel_source_hash()
    assert len(profiling.kernel_source_hash()) == 16


def test_dominant_depth():
    """The depth most passes run at when T sweeps are split into passes whose
    depths differ by at most one (the library's pass planner)."""
    import bench
    assert bench.dominant_depth(50, 8) == 6      # 6 passes of 6, 2 of 7
    assert bench.dominant_depth(50, 7) == 7      # 6 of 7, 1 of 8
    assert bench.dominant_depth(100, 25) == 4
    assert bench.dominant_depth(32, 8) == 4
    assert bench.dominant_depth(11, 3) == 4      # 4, 4, 3
