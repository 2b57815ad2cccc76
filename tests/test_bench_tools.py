"""Host logic of bench.py's block-size table (no GPU): a synthetic kernel
trace and step file with known durations give the expected per-size rows,
and launches past the last traced step (end-time gate) are left out."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _write(tmp_path, runs):
    """runs: per precision, a list of (n_act, front_us, pair_us, rc_us); each
    run gets one extra untraced step (a no-op past the end time)."""
    rows, steps, t = [], [], 0
    for prec, run in enumerate(runs):
        for k, (n_act, f, p, r) in enumerate(run + [(0, 1.0, 1.0, 1.0)]):
            for name, d in ((f"void nb::blk_front_kernel<{prec}>(int)", f),
                            (f"void nb::blk_step_kernel<{prec}, false>(nb::ForceArgs)", p),
                            ("nb::blk_reduce_correct_kernel(nb::ReduceArgs, nb::CorrectArgs)", r)):
                rows.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + int(d * 1000)})
                t += int(d * 1000) + 500
            if k < len(run):
                steps.append({"mode": "block", "step": k + 1, "n_act": n_act})
    tr = tmp_path / "trace.csv"
    with open(tr, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerows(rows)
    sj = tmp_path / "steps.jsonl"
    sj.write_text("".join(json.dumps(s).replace('"mode":"block"', '"mode": "block"') + "\n" for s in steps))
    return str(tr), str(sj)


def test_block_size_table(tmp_path):
    import bench
    fp32 = [(1, 7.0, 5.0, 5.0), (1, 9.0, 7.0, 3.0), (100, 7.0, 20.0, 6.0)]
    ds = [(20000, 6.0, 1000.0, 70.0)]
    tr, sj = _write(tmp_path, [fp32, ds])
    text = bench.block_size_table(tr, sj, n_total=1000)
    lines = text.splitlines()
    assert lines[0].startswith("fp32: 3 traced block steps")
    one = next(l for l in lines if l.split()[0] == "1-1").split()
    assert one[1:5] == ["2", "8.00", "6.00", "4.00"]          # means of the two 1-particle steps
    assert float(one[5]) == round(2 * 1000 / 12.0 / 1e3, 1)   # 2 x 1000 interactions in 12 us
    mid = next(l for l in lines if l.split()[0] == "64-255").split()
    assert mid[1:5] == ["1", "7.00", "20.00", "6.00"]
    i = lines.index(next(l for l in lines if l.startswith("ds:")))
    big = next(l for l in lines[i:] if l.split()[0] == "16384-").split()
    assert big[1:5] == ["1", "6.00", "1000.00", "70.00"]
    assert float(big[5]) == round(20000 * 1000 / 1000.0 / 1e3, 1)
