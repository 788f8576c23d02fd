"""The rocprofv3 summariser on small synthetic CSV files (CPU)."""
from paper_1901_01047_amd import profsum


def test_trace_summary_separates_empty_dispatches(tmp_path):
    p = tmp_path / "kernel_trace.csv"
    rows = ["Kind,Kernel_Name,Start_Timestamp,End_Timestamp"]
    t = 0
    for d in (100_000, 2_000, 120_000, 1_500):       # ns: two working, two empty dispatches
        rows.append(f"KERNEL_DISPATCH,k_fold<double>,{t},{t + d}")
        t += d + 10
    rows.append(f"KERNEL_DISPATCH,k_accept<double>,{t},{t + 50_000}")
    p.write_text("\n".join(rows) + "\n")
    s = {r["kernel"]: r for r in profsum.trace_summary(str(p), noop_us=3.0)}
    f = s["k_fold<double>"]
    assert f["calls"] == 4 and f["noop_calls"] == 2
    assert abs(f["avg_active_us"] - 110.0) < 1e-9
    assert abs(f["total_ms"] - 0.2235) < 1e-9
    assert s["k_accept<double>"]["noop_calls"] == 0
    assert "| `k_fold<double>` | 4 | 2 | 110.00 |" in profsum.trace_table(profsum.trace_summary(str(p)))


def test_pmc_summary_per_dispatch(tmp_path):
    p = tmp_path / "counter_collection.csv"
    p.write_text("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
                 "1,k_fold<double>,FETCH_SIZE,10\n1,k_fold<double>,FETCH_SIZE,5\n"
                 "2,k_fold<double>,FETCH_SIZE,20\n3,k_gather<double>,FETCH_SIZE,99\n")
    r = profsum.pmc_summary(str(p), r"k_fold", "FETCH_SIZE")
    assert r["dispatches"] == 2 and r["median"] == 17.5 and r["mean"] == 17.5
