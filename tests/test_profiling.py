"""Host logic of the counter summaries: which dispatch scales the HBM byte counters, and
the bytes per launch they give (no GPU; synthetic rocprofv3 counter tables)."""
import csv
import json

from paper_1910_08535_amd import profiling

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
MIB256 = 256 * 1024   # KiB


def _write(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for did, grid, name, val in rows:
            w.writerow({"Dispatch_Id": did, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": val})


def _tables(tmp_path):
    """A run: the 256 MiB copy probe first (a fill, then three copies), then a 1 GiB fill of
    a later input (an elementwise kernel with more traffic than the probe), then the
    kernel of interest at two grid sizes."""
    fetch = [(1, 256, "vectorized_elementwise_kernel<FillFunctor>", 17.0)]
    write = [(1, 256, "vectorized_elementwise_kernel<FillFunctor>", MIB256)]
    for d in (2, 3, 4):
        fetch.append((d, 1024, "__amd_rocclr_copyBuffer", MIB256 / 2))   # counts half
        write.append((d, 1024, "__amd_rocclr_copyBuffer", MIB256))
    fetch.append((5, 4096, "distribution_elementwise_grid_stride_kernel", 10.0))
    write.append((5, 4096, "distribution_elementwise_grid_stride_kernel", 4 * MIB256))
    for d in range(6, 12):
        grid = "74304" if d % 3 else "999"
        fetch.append((d, grid, "iga::apply2d_kernel<2, 8, 3, true>", 4600.0))
        write.append((d, grid, "iga::apply2d_kernel<2, 8, 3, true>", 17000.0))
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    return str(fp), str(wp)


def test_probe_is_the_first_copies(tmp_path):
    fp, wp = _tables(tmp_path)
    assert profiling._probe_value(fp, "FETCH_SIZE") == MIB256 / 2
    # the later 1 GiB fill is not the probe
    assert profiling._probe_value(wp, "WRITE_SIZE") == MIB256


def test_traffic_scales_by_the_probe(tmp_path):
    fp, wp = _tables(tmp_path)
    rec = profiling.traffic(fp, wp, "apply2d_kernel<2, 8, 3, true>@74304", 256, "t", "cmd",
                            out_dir=str(tmp_path))
    assert rec["grid_size"] == "74304" and rec["dispatches"] == [4, 4]
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["fetch_bytes_per_launch"] == 4600.0 * 1024 * 2
    assert rec["write_bytes_per_launch"] == 17000.0 * 1024
    assert json.loads((tmp_path / "traffic_t.json").read_text())["bytes_per_launch"] == rec["bytes_per_launch"]
