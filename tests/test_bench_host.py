"""Host-side pieces of bench.py: the CPU-baseline leg runs the oracle's step on a tiny workload and
reports what the line needs (rate, threads, sample).  CPU only."""
import numpy as np

import bench
import synth


def test_cpu_baseline_runs_the_oracle_step_on_a_small_plan():
    c = synth.make_config("er64", seed=0)
    F, L, alphas = c["F"], c["L"], c["alphas"]
    X = synth.real_signals((len(alphas), F.shape[0], 8), np.random.default_rng(2)).astype(np.float32)
    out = bench.cpu_baseline(F, alphas, L, X, budget_s=0.5, chunk=4, one_thread_orders=4)
    assert out["kind"] == "oracle" and out["unit"] == "updates/s"
    assert out["value"] > 0 and out["seconds"] > 0
    assert out["cores"] >= 1 and out["affinity_cores"] >= 1
    assert isinstance(out["cpu_model"], str) and out["cpu_model"]
    assert out["one_thread"]["orders"] == 4 and out["one_thread"]["value"] > 0
    assert "orders of the same workload" in out["sample"]


def test_algorithmic_byte_counts():
    # per order 8 N^2 written plus (L+2) 4 N^2 of stack and projector read once per call
    assert bench.update_algorithmic_bytes(4096, 32, 256) == 256 * 8 * 4096 ** 2 + 34 * 4 * 4096 ** 2
    assert bench.apply_algorithmic_bytes(4096, 64, 256) == 256 * (8 * 4096 ** 2 + 12 * 4096 * 64)


def test_stored_traffic_counters_belong_to_the_committed_kernels():
    # the HBM byte counts the line reports were taken on these exact sources; a kernel edit without
    # new counter runs must show up here (the bench would then report the traffic as null)
    assert bench.UPDATE_TRAFFIC["source_sha256"] == bench.update_source_digest()
    assert bench.DIRECT_TRAFFIC["source_sha256"] == bench.source_digest("direct.hip")
    # and they sit just above the algorithmic bytes: no kernel re-reads its operands
    alg = bench.update_algorithmic_bytes(4096, 32, 256)
    assert 1.0 <= bench.update_traffic() / alg < 1.1
    d = bench.DIRECT_TRAFFIC
    d_alg = 33 * 4 * 4096 ** 2 + 12 * 4096 * d["ncols"]    # (L+1) 4N^2 of stack and P, 12 N per column
    assert 0.99 <= (d["fetch_bytes"] + d["write_bytes"]) / d_alg < 1.1
