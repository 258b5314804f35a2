"""profile_summary turns rocprofv3 CSV files into the tables kept under
profiles/ (host only: it reads CSV text)."""
import csv

from paper_0908_2654_amd import profile_summary as ps


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def test_markers_table_sorted_and_in_ms(tmp_path):
    p = tmp_path / "marker_api_stats.csv"
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
           "StdDev"]
    _write(p, hdr, [["V-cycles", 3, 6_000_000, 2_000_000, 20, 1, 1, 0],
                    ["rh_implicit_step", 1, 30_000_000, 30_000_000, 80, 1, 1, 0]])
    lines = ps.markers_table(str(p)).splitlines()
    assert lines[2] == "| rh_implicit_step | 1 | 30.000 | 30.0 |"
    assert lines[3] == "| V-cycles | 3 | 2.000 | 6.0 |"


def test_stats_table_shares(tmp_path):
    p = tmp_path / "kernel_stats.csv"
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
           "StdDev"]
    _write(p, hdr, [["void rh::(anonymous namespace)::k_a<float>(int)", 4, 3_000_000, 750_000,
                     75, 1, 1, 0],
                    ["k_b(double*)", 1, 1_000_000, 1_000_000, 25, 1, 1, 0]])
    lines = ps.stats_table(str(p)).splitlines()
    assert lines[2] == "| `k_a<float>` | 4 | 0.7500 | 3.0 | 75.0 |"
    assert lines[3] == "| `k_b` | 1 | 1.0000 | 1.0 | 25.0 |"
