"""The measurement code of bench.py: the algorithmic byte model of one
BiCGSTAB iteration, the scaling of counter-measured traffic by the plain copy
kernel, the kernel-source check that keeps a stale traffic record out of the
bench line, and the kernel-trace summary's iteration time.  CPU only; the
counter and trace files are written here."""
import csv
import json

import pytest

import bench


def test_kernel_bytes_per_node_model():
    # the byte model stated per node: p/v moves 4 B per index, 8 B per
    # per-node weight and 88 B of vectors; s/t the same indices and weights
    # and 40 B of vectors.  Regular nodes on the shared lattice row carry no
    # weights of their own.
    buckets = [(0, 5, 100), (1, 12, 10), (2, 30, 3)]
    N = 113
    shared = 5 * 100
    per_node_pv = [4 * 5 + 88] * 100 + [(4 + 8) * 12 + 88] * 10 + [(4 + 8) * 30 + 88] * 3
    per_node_st = [4 * 5 + 40] * 100 + [(4 + 8) * 12 + 40] * 10 + [(4 + 8) * 30 + 40] * 3
    assert bench.kernel_bytes(buckets, N, "bicg_pv", shared) == sum(per_node_pv)
    assert bench.kernel_bytes(buckets, N, "bicg_st", shared) == sum(per_node_st)
    assert bench.kernel_bytes(buckets, N, "iteration", shared) == sum(per_node_pv) + sum(per_node_st)
    # without the shared row every regular node carries its 5 weights, in both kernels
    assert (bench.kernel_bytes(buckets, N, "iteration") - bench.kernel_bytes(buckets, N, "iteration", shared)
            == 2 * 8 * 5 * 100)
    with pytest.raises(ValueError):
        bench.kernel_bytes(buckets, N, "apply")


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=i, Kernel_Name=name, Counter_Name=counter, Counter_Value=kib))


def _bench_line(path, domains, nodes, rows_matvec, alg):
    line = dict(config=dict(domains=domains, nodes=nodes, workload="w"),
                roofline=dict(kernel="k", node_rows_matvec=rows_matvec, bytes_per_launch=alg))
    open(path, "w").write("a log line\n" + json.dumps(line) + "\n")


def test_pmc_summary_one_domain(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(out))
    copy_kib = 2.0 ** 31 / 1024 / 2      # the copy kernel's fetch counter reads half its bytes: scale 2
    fetch = [("k_stream_copy", copy_kib)] + [("k_bicg_pv<2, 8, true, true>", v) for v in (1.0, 10.0, 12.0, 11.0)] \
        + [("k_bicg_st<2, true, true>", v) for v in (2.0, 6.0, 5.0, 7.0)]
    write = [("k_stream_copy", 2.0 ** 31 / 1024)] + [("k_bicg_pv<2, 8, true, true>", 3.0)] * 4 \
        + [("k_bicg_st<2, true, true>", 1.0)] * 4
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    _bench_line(tmp_path / "b.json", 1, 1000, 0, 100000.0)
    bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.json"), "c2")
    rec = json.load(open(out))
    assert rec["copy_fetch_scale"] == pytest.approx(2.0) and rec["copy_write_scale"] == pytest.approx(1.0)
    # one domain: the median of the busy (upper) half of the launches
    assert rec["fetch_bytes_pv"] == pytest.approx(2.0 * 1024 * 11.5)
    assert rec["fetch_bytes_st"] == pytest.approx(2.0 * 1024 * 6.5)
    assert rec["write_bytes_pv"] == pytest.approx(1024 * 3.0) and rec["write_bytes_st"] == pytest.approx(1024.0)
    total = 2048 * 11.5 + 2048 * 6.5 + 1024 * 3.0 + 1024.0
    assert rec["hbm_bytes_per_iteration"] == pytest.approx(total)
    assert rec["over_algorithmic"] == pytest.approx(total / 100000.0)
    assert rec["kernel_source_sha256"] == bench.kernel_source_sha()


def test_pmc_summary_many_domains_per_full_iteration(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(out))
    fetch = [("k_stream_copy", 2.0 ** 31 / 1024)] + [("k_bicg_pv", 4.0)] * 6 + [("k_bicg_st", 2.0)] * 6
    write = [("k_stream_copy", 2.0 ** 31 / 1024)] + [("k_bicg_pv", 1.0)] * 6 + [("k_bicg_st", 1.0)] * 6
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write)
    # 3 full-iteration equivalents: 2 N matvec rows each
    _bench_line(tmp_path / "b.json", 8, 500, 3 * 2 * 500, 1.0)
    bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "b.json"), "c3")
    rec = json.load(open(out))
    assert rec["fetch_bytes_pv"] == pytest.approx(6 * 4.0 * 1024 / 3)
    assert rec["fetch_bytes_st"] == pytest.approx(6 * 2.0 * 1024 / 3)
    assert rec["write_bytes_pv"] == pytest.approx(6 * 1024 / 3)


def test_traffic_record_needs_the_measured_kernel_sources(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda w: str(path))
    assert bench.traffic_record("c3") is None                     # no record
    json.dump(dict(kernel_source_sha256="0" * 64, hbm_bytes_per_iteration=1.0), open(path, "w"))
    assert bench.traffic_record("c3") is None                     # measured on other kernels
    json.dump(dict(kernel_source_sha256=bench.kernel_source_sha(), hbm_bytes_per_iteration=1.0), open(path, "w"))
    assert bench.traffic_record("c3")["hbm_bytes_per_iteration"] == 1.0


def test_trace_summary_iteration_from_batch_spans(tmp_path):
    # a synthetic kernel trace: an autotuner candidate build with a time step,
    # then the timed build, its right-hand side and three batches of four
    # iterations; the third batch's p/v launches return at once (queued past
    # convergence), so only the first two count as full batches
    ns = lambda us: int(us * 1000)
    rows = []

    def k(name, start_us, dur_us, grid=256):
        rows.append(dict(Kernel_Name=f"void hsm::(anonymous namespace)::{name}(hsm::SimArgs)", Grid_Size_X=grid,
                         Start_Timestamp=ns(start_us), End_Timestamp=ns(start_us + dur_us)))

    k("k_bbox_part", 0, 1)
    k("k_predict<2, double>", 5, 1)
    k("k_bbox_part", 100, 1)
    k("k_predict<2, double>", 105, 1)
    k("k_rhs<2, double>", 110, 2)               # the first batch starts where this ends: 112 us
    t = 112.0
    for per_it, pv_us in ((20.0, 5.0), (25.0, 6.0), (4.0, 1.0)):
        for j in range(4):
            k("k_bicg_pv<2, 8, true, true>", t + j * per_it, pv_us)
            k("k_bicg_st<2, true, true>", t + j * per_it + pv_us, 2.0)
        t += 4 * per_it
        k("k_chunk_end", t - 1.0, 1.0, grid=1024)    # ends at t
    trace = tmp_path / "trace.csv"
    with open(trace, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        for r in rows[::-1]:                    # any order: the summary sorts by start time
            w.writerow(r)
    stats = tmp_path / "stats.csv"
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow(dict(Name="k_bicg_pv<2, 8, true, true>", Calls=12, AverageNs=4000, Percentage=50.0))
    out = tmp_path / "summary.txt"
    bench.trace_summary(str(trace), str(stats), 0, 1, "cmd", str(out))
    text = out.read_text()
    assert "full batches of 4 iterations: 2" in text
    assert "mean iteration time (chunk_end-to-chunk_end span / 4): 22.50 us" in text
    # every batch, idle or not: 80 + 100 + 16 us
    assert "all batches (the last of each solve partly idle; with many domains, each domain stops on its own): " \
           "3, total 0.196 ms" in text
    assert "k_bicg_pv<2, 8, true, true> [grid 256]" in text
