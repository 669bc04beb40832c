"""Host logic of the serving summary: counts, percentiles over all requests with capped and failed
solves counted as never reaching the target, and percentiles over the converged ones."""
import math

from paper_1810_07803_amd import hrlb, serve


def _rec(k, state, status, arrival, admit, done):
    r = dict(index=k, state=state, status=status, arrival=arrival, admit=admit)
    if done is not None:
        r["done"] = done
    return r


def test_counts_and_percentiles_with_capped_requests():
    recs = [_rec(k, "done", hrlb.HRLB_OK, 0.1 * k, 0.1 * k + 0.05, 0.1 * k + 1.0 + k) for k in range(8)]
    recs.append(_rec(8, "done", hrlb.HRLB_NOT_CONVERGED, 0.0, 0.1, 50.0))
    recs.append(_rec(9, "failed", -4, 0.0, 0.1, None))
    s = serve.latency_summary(recs)
    assert (s["requests"], s["finished"], s["converged"], s["capped"], s["failed"], s["unfinished"]) == (10, 9, 8, 1, 1, 0)
    # times to steady of the converged requests: 1 + k for k = 0..7; the two others never arrive
    assert s["p50_time_to_steady_s"] == 5.0
    assert s["p99_time_to_steady_s"] is None
    assert math.isclose(s["p50_time_to_steady_converged_s"], 4.0)
    assert math.isclose(s["p99_time_to_steady_converged_s"], 8.0)
    # arrival -> result over the finished requests includes the capped one
    assert math.isclose(s["p99_arrival_to_result_s"], 50.0)
    assert math.isclose(s["p50_admit_to_result_s"], 4.95)


def test_all_converged_gives_the_same_percentiles_both_ways():
    recs = [_rec(k, "done", hrlb.HRLB_OK, 0.0, 0.0, 1.0 + k) for k in range(32)]
    s = serve.latency_summary(recs)
    assert s["p50_time_to_steady_s"] == s["p50_time_to_steady_converged_s"]
    assert s["p99_time_to_steady_s"] == s["p99_time_to_steady_converged_s"] == 32.0
