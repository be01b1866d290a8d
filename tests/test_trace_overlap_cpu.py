"""The kernel-trace overlap tool on a small hand-made trace (host only): dispatches of two
queues, shared time merged across partners, dispatches of one queue alone left out."""
import csv

from paper_2507_15703_amd import trace_overlap


def _write(path, rows):
    cols = ["Kind", "Agent_Id", "Queue_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for q, name, s, e in rows:
            w.writerow({"Kind": "KERNEL_DISPATCH", "Agent_Id": "Agent 1", "Queue_Id": q, "Kernel_Name": name,
                        "Start_Timestamp": s, "End_Timestamp": e})


def test_overlap_of_two_queues(tmp_path):
    p = tmp_path / "trace.csv"
    _write(p, [
        (1, "void cmbx::k_pass_x<float, 512, 8, 0>(cmbx::cpx<float>*)", 0, 10_000),
        (2, "void cmbx::k_pass_y<float, 512, 16, 1>(cmbx::cpx<float>*)", 5_000, 20_000),
        (1, "void cmbx::k_gather<float, 4>(float const*)", 12_000, 15_000),
        (1, "void cmbx::k_pass_x<float, 512, 8, 0>(cmbx::cpx<float>*)", 18_000, 30_000),
        (1, "void cmbx::k_pass_x<float, 512, 8, 0>(cmbx::cpx<float>*)", 40_000, 50_000),
        (2, "cmbx::(anonymous namespace)::k_hybrid_columns<float, 16>(int)", 41_000, 42_000),
    ])
    rows = trace_overlap.load(str(p))
    assert {r[3] for r in rows} == {"k_pass_x<float, 512, 8, 0>", "k_pass_y<float, 512, 16, 1>",
                                   "k_gather<float, 4>", "k_hybrid_columns<float, 16>"}
    out = trace_overlap.overlap(rows, ["k_pass_x", "k_pass_y"])
    x = out["k_pass_x"]
    # [0, 10) meets y over [5, 10); [18, 30) over [18, 20); [40, 50) meets the hybrid kernel
    assert x["dispatches"] == 3
    assert abs(x["busy_us"] - 32.0) < 1e-9
    assert abs(x["shared_us"] - (5.0 + 2.0 + 1.0)) < 1e-9
    assert x["with"] == {"k_pass_y<float, 512, 16, 1>": 7.0, "k_hybrid_columns<float, 16>": 1.0}
    y = out["k_pass_y"]
    # y [5, 20) meets x [5, 10), the gather [12, 15) and x [18, 20): merged 10 of its 15 us
    assert y["dispatches"] == 1
    assert abs(y["shared_us"] - 10.0) < 1e-9 and abs(y["shared_frac"] - 10.0 / 15.0) < 1e-12


def test_one_queue_alone_counts_nothing(tmp_path):
    p = tmp_path / "trace.csv"
    _write(p, [(1, "void cmbx::k_pass_x<float, 512, 8, 0>(int)", 0, 10), (1, "void cmbx::k_gather<float, 4>(int)", 10, 20)])
    out = trace_overlap.overlap(trace_overlap.load(str(p)), ["k_pass_x", "k_gather"])
    assert out["k_pass_x"]["dispatches"] == 0 and out["k_gather"]["shared_frac"] == 0.0
