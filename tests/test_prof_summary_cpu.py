"""The rocprofv3 summaries keep exactly the launches the library timed: the dispatches
between the k_profile_mark kernels that t2s_profile_enable issues (synthetic trace
database and counter CSV, no GPU)."""

import csv
import os
import sqlite3

import pytest

from paper_1809_04195_amd import prof_summary as PS


def _db(path, seq):
    db = sqlite3.connect(path)
    db.execute("create table kernels (name text, start integer, end integer)")
    db.executemany("insert into kernels values (?, ?, ?)", seq)
    db.commit()
    db.close()


def test_stats_window_and_after(tmp_path):
    seq, t = [], 0
    for name in ["k_passB<384, 5>", "k_profile_mark()", "k_passB<384, 5>", "k_passA<384, 1>", "k_passB<384, 5>",
                 "k_profile_mark()", "k_passB<384, 5>", "k_profile_mark()", "k_llr<5, 8, 0>", "k_profile_mark()"]:
        dur = 10 if "mark" in name else (100 if "passB" in name else 50)
        seq.append((name, t, t + dur))
        t += dur + 5
    path = os.path.join(tmp_path, "run_results.db")
    _db(path, seq)
    rows = {r[0]: r for r in PS._stats_rows(str(tmp_path), window=1)}
    assert set(rows) == {"k_passB<384, 5>", "k_passA<384, 1>"}
    assert rows["k_passB<384, 5>"][1] == 2 and rows["k_passB<384, 5>"][3] == 100
    rows2 = {r[0]: r for r in PS._stats_rows(str(tmp_path), window=2)}
    assert set(rows2) == {"k_llr<5, 8, 0>"}
    every = {r[0]: r for r in PS._stats_rows(str(tmp_path))}
    assert every["k_passB<384, 5>"][1] == 4 and "k_profile_mark()" not in every
    after = {r[0]: r for r in PS._stats_rows(str(tmp_path), after="k_passB:3")}
    assert after["k_passB<384, 5>"][1] == 2
    with pytest.raises(ValueError):
        PS._stats_rows(str(tmp_path), window=3)


def test_counters_window(tmp_path):
    path = os.path.join(tmp_path, "run_counter_collection.csv")
    names = ["k_passB<384, 5>(x)", "k_profile_mark()", "k_passB<384, 5>(x)", "k_passC<384, 2, 1, 2>(x)",
             "k_profile_mark()", "k_passB<384, 5>(x)"]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"])
        for i, n in enumerate(names):
            w.writerow([i + 1, n, "FETCH_SIZE", 1000.0 * (i + 1), 100 * i, 100 * i + 40])
    fam = PS.read_counters(path, window=1)
    assert set(fam) == {"pass_b", "pass_c"}
    assert fam["pass_b"]["n"] == 1 and fam["pass_b"]["FETCH_SIZE"] == 3000.0
    assert PS.read_counters(path)["pass_b"]["n"] == 3


def test_family_names():
    assert PS.family("void t2s::k_passC<384, 1, 1, 2>(t2s::ClassArgs, int)") == "passC_adjoint"
    assert PS.family("void t2s::k_passC<384, 2, 1, 2>(t2s::ClassArgs, int)") == "pass_c"
    assert PS.family("t2s::k_llr_finalize(t2s::ClassArgs, int)") == "llr_finalize"
    assert PS.family("void t2s::k_llr<5, 8, 0>(...)") == "llr_admm"
